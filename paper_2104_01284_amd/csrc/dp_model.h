// Device-side problem parameters and the FP64 stage model of the eco-driving
// DP (Zhu et al., ECC 2021, Sec. III).  Shared by the kernels of this library
// only; host code fills DevInst once per plan.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecodp {

constexpr int kSortBins = 4096;   // speed-cell bins of the per-node control sort

// Per-instance constants, passed to kernels by value.
struct DevInst {
    int N, n_v, n_s, n_t, n_e, n_m, n_u;
    int wait;            // DP_WAIT_AT_RED
    int zero_row;        // index of the v = 0 speed node, or -1
    double ds;
    double v_lo, s_lo;
    double v_hi, s_hi, t_f;
    double hv, hs, ht, he, hm;
    double e_lo, m_lo;
    double M, CdA, Crr, wt, wsoc;
    double g, rho, rw, ig, eta, etam, Cnom, Voc0, Voc1, Rb, amin, amax, xiref, Jinf;
    double peng, pbsg;           // engine and BSG power caps [W] (Eq. 7e-f), 0 = none
    double q[6];
    double v0, soc0, t0_abs;
    const double *cosa, *sina;   // [N] grade trigonometry (host FP64)
    const double *vmax;          // [N+1]
    const int *light_of_stage;   // [N+1]: signal index at stage k or -1
    const double *l_cycle, *l_red, *l_off, *l_yel;
    const float *terminal_V;     // optional
};

// Compact per-(speed node, control) data of one stage, FP64-derived.
struct StageEntry {
    float c;       // stage cost (mf + w_t) dt
    float fv, gv;  // speed fraction and 1 - fraction (each rounded from FP64)
    float ft, gt;  // time fraction of the per-step advance dt / h_t
    int16_t iv;    // lower speed cell in [0, n_v - 2]; -1 = infeasible pair
    int16_t dtc;   // whole time cells advanced
};

// Stage data of one (speed node, control) in the order the grouped sweep
// visits it: ascending next-stage speed cell, ascending control inside a cell.
struct SortedEntry {
    float c;
    float fv, gv;  // speed weights of the upper and lower successor cell
    float ft;      // time fraction inside the successor cell
    float rt;      // ft / gt: the time lerp is gt (V(t) + rt V(t+1)), gt folded into the SoC weights
    int32_t iv;    // lower speed cell of the successor (>= 0: infeasible pairs are dropped)
    int32_t dtc;   // whole time cells advanced
    int32_t u;     // control index a * n_m + b
};

// Per-(speed node, control, SoC node) battery coordinate.
struct BatEntry {
    int32_t jx;    // lower SoC cell in [0, n_s - 2]; -1 = infeasible
    float fx, gx;
};

// Scalars the grouped sweep needs (kept small: everything here lives in SGPRs).
struct SweepArgs {
    int n_v, n_t, n_s, n_u, zero_row, wait;
    float Jinf;
    double v_lo, hv;
    const double *vmax;
};

// Per-(signal, time node) data, host FP64.
struct TLEntry {
    int32_t red;   // 1 if the node's absolute time is in a red phase
    int32_t wc;    // wait: lower time cell of t_m + tau; -1 if beyond t_f
    double wf;     // wait: fraction
    double tau;    // wait: time until green [s]
    float wcost;   // w_t * tau rounded to FP32
    float wf32, wg32;
    int32_t ncyc;  // dtau/dC of the wait: whole cycles n in t_abs - O = n C + phase, + 1 in yellow
    int32_t yel;   // 1 if the node's absolute time is in a yellow phase
    int32_t pad;
    double ys;     // yellow: time since yellow began [s]
};

// 1 when a vehicle at speed v has to stop at the signal of entry t (Eq. 8
// with the yellow rule of Sec. III): in red, or in yellow once more time has
// passed since yellow began than v / (2 b), b = -a_min the braking limit (it
// was beyond its critical braking distance v^2 / (2 b) when yellow began).
__device__ __host__ inline bool tl_stop(const TLEntry &t, double v, double amin)
{
#pragma clang fp contract(off)
    return t.red || (t.yel && t.ys > v / (2.0 * -amin));
}

// Value of waiting at a signal (the waiting cost plus the next stage's values
// lerped at the time reached when green begins, pw pointing at the lower time
// cell).  Written with explicit fused steps so that every kernel forming it
// (sweep, control-slice combine, simple sweep) rounds the same way.
__device__ __forceinline__ float wait_value(const TLEntry &t, const float *pw)
{
    return t.wcost + fmaf(t.wg32, pw[0], t.wf32 * pw[1]);
}

// One (instance, stage) of the grouped sweep.  Buffer positions are byte
// offsets from the J, pi and scratch pointers of the call, so one table built
// with the plan serves every call.
struct StageJob {
    int inst;              // index of the instance's parameter block
    int k;                 // stage
    int jt;                // SoC rows per workgroup
    int ntiles;            // SoC tiles
    int nsplit;            // control slices per (speed node, tile)
    int H;                 // bound on the SoC-cell shift of one step
    int rw;                // staged SoC rows per plane (jt + 2H + 2)
    int nitems;            // n_v * ntiles * nsplit sweep items
    int tl;                // offset (entries) of the stage's signal table, -1 = none
    int pad;
    long long jn, jk, pik;                 // J_{k+1}, J_k (J buffer), pi_k (pi buffer)
    long long st, nf, rec, pv, pu;         // stage data and partial results (scratch)
    long long pw;                          // battery power and time step per sorted control (scratch)
};

// Launch-wide pointers of a set of jobs.  Jn / Jk / pik, when set, replace the
// J and pi buffers of a single job (an isolated stage on caller slabs).
struct StageBase {
    const DevInst *insts;
    const StageJob *jobs;
    char *J;
    char *pi;
    char *scr;
    const TLEntry *tl;
    const float *Jn;
    float *Jk;
    int16_t *pik;
    unsigned long long *count;   // per instance: state-control evaluations the sweep executed
    int *err;                    // plan's device error word (kDevErr* bits)
};

// Bits of the plan's device error word (sticky until read by the host).
constexpr int kDevErrCellOffset = 1;   // a SoC cell offset did not fit the records' int8 field
constexpr int kDevErrWait = 2;         // a persistent sweep gave up waiting for a stage
constexpr int kDevErrNegative = 4;     // a device terminal_V value was negative (costs must not be)

// One (instance, stage) job of the persistent sweep: the stage job, the items
// of the instance's later stages that must be counted before it starts, and
// its first item in its XCD queue.
struct PJob {
    StageJob j;
    int need;
    int item0;
    int pad[2];
};

// Queues of one persistent sweep launch: per XCD a range of jobs and its item
// count; claim counters per XCD and done counters per instance (scratch,
// cleared before the launch).
struct PersistQueues {
    const PJob *jobs;
    const int *xjb;        // [n_xcd + 1] job bounds of the XCD queues
    const int *xtot;       // [n_xcd] items of each XCD queue
    int *claim;            // [n_xcd]
    int *done;             // [n_inst] items counted per instance
    int *err;              // the plan's device error word
    int n_xcd;
    int stall;             // test hook: each queue's first job waits for a count never reached
    long long spin_limit;  // polls (each followed by a short sleep) before a wait gives up
};

// Result of the continuous one-step model for (stage k, speed v, control).
struct PT {
    double v1, acc, dt, cost, mf, Pb, q, Ftr, Froad, cosa, sina;
    int st;        // 1 accel bound, 2 speed limit, 4 zero mean speed, 16 torque limit
};

// Eq. 5a (constant force over the step), Eq. 2, Eq. 1 and the BSG power
// demand.  FP64 without contraction so that cells and feasibility match an
// IEEE double evaluation of the same expressions.
__device__ __host__ inline PT powertrain(const DevInst &P, int k, double v, int a, int b)
{
#pragma clang fp contract(off)
    PT p;
    const double Te = P.e_lo + a * P.he;
    const double Tm = P.m_lo + b * P.hm;
    p.cosa = P.cosa[k];
    p.sina = P.sina[k];
    p.Ftr = P.eta * (Te + Tm) * P.ig / P.rw;
    p.Froad = P.M * P.g * (P.Crr * p.cosa + p.sina) + 0.5 * P.rho * P.CdA * v * v;
    p.q = v * v + 2.0 * P.ds * (p.Ftr - p.Froad) / P.M;
    p.st = 0;
    if (p.q > 0.0) {
        p.v1 = sqrt(p.q);
        p.acc = (p.Ftr - p.Froad) / P.M;
    } else {
        p.v1 = 0.0;                       // stops inside the step
        p.acc = -v * v / (2.0 * P.ds);
    }
    if (p.acc < P.amin || p.acc > P.amax) p.st |= 1;
    if (p.v1 > P.vmax[k + 1]) p.st |= 2;
    const double vs = v + p.v1;
    if (!(vs > 0.0)) {
        p.st |= 4;
        p.dt = 1.0e300;
    } else {
        p.dt = 2.0 * P.ds / vs;
    }
    double mf = 0.0;
    if (Te != 0.0) {
        mf = P.q[0] + P.q[1] * v + P.q[2] * Te + P.q[3] * v * v + P.q[4] * v * Te + P.q[5] * Te * Te;
        if (mf < 0.0) mf = 0.0;
    }
    p.mf = mf;
    p.cost = (mf + P.wt) * p.dt;
    const double w = v * P.ig / P.rw;
    const double Pm = Tm * w;
    p.Pb = Pm >= 0.0 ? Pm / P.etam : Pm * P.etam;
    // Eq. 7e-f: the torque a power cap allows at the step's initial crank speed
    if (P.peng > 0.0 && Te * w > P.peng) p.st |= 16;
    if (P.pbsg > 0.0 && fabs(Tm) * w > P.pbsg) p.st |= 16;
    return p;
}

// Zeroth-order battery: the current drawn for power Pb at SoC xi, or false if
// Pb exceeds Voc^2 / (4R).
__device__ __host__ inline bool battery_current(const DevInst &P, double Pb, double xi, double &I)
{
#pragma clang fp contract(off)
    const double Voc = P.Voc0 + P.Voc1 * xi;
    const double D = Voc * Voc - 4.0 * P.Rb * Pb;
    if (D < 0.0) return false;
    I = 2.0 * Pb / (Voc + sqrt(D));
    return true;
}

// Lower cell and fraction of an index coordinate r in [0, n-1]: c = min(floor r, n-2).
__device__ __host__ inline void cell_of(double r, int n, int &c, double &f)
{
    const double fl = floor(r);
    c = (int)fl;
    if (c > n - 2) c = n - 2;
    f = r - c;
}

}  // namespace ecodp
