// FP64 kernels that follow the stored policy: the forward rollout from x0 and
// the fixed-policy adjoint dV_0/dtheta (forward sweep of the occupancy
// measure, i.e. the transpose of the trilinear interpolation, stage by stage).
#include "dp_internal.h"

namespace ecodp {

// 1 when a vehicle at speed v has to stop at signal L at relative time t_rel
// (Eq. 8, with the yellow rule of Sec. III: red, or yellow once more time has
// passed since yellow began than v / (2 b), b = -a_min), with tau the time
// until green.
__device__ inline bool must_stop(const DevInst &P, int L, double t_rel, double v, double &tau)
{
#pragma clang fp contract(off)
    const double C = P.l_cycle[L], R = P.l_red[L], Y = P.l_yel[L];
    double x = fmod(P.t0_abs + t_rel - P.l_off[L], C);
    if (x < 0.0) x += C;
    tau = 0.0;
    if (x < R) {
        tau = R - x;
        return true;
    }
    if (Y > 0.0 && x >= C - Y && x - (C - Y) > v / (2.0 * -P.amin)) {
        tau = (C - x) + R;
        return true;
    }
    return false;
}

// Control at an off-grid state: among the bracketing nodes with positive
// weight and a stored control (>= 0), the largest weight; equal weights go to
// the lowest linear node index; -1 if none.
__device__ int policy_lookup(const DevInst &P, const int16_t *pik, double v, double xi, double t, int &oog)
{
#pragma clang fp contract(off)
    double r[3] = {(v - P.v_lo) / P.hv, (xi - P.s_lo) / P.hs, t / P.ht};
    const int n[3] = {P.n_v, P.n_s, P.n_t};
    int c[3];
    double f[3];
    for (int d = 0; d < 3; d++) {
        if (r[d] < 0.0) {
            r[d] = 0.0;
            oog = 1;
        }
        if (r[d] > n[d] - 1) {
            r[d] = n[d] - 1;
            oog = 1;
        }
        cell_of(r[d], n[d], c[d], f[d]);
    }
    double bw = -1.0;
    long bn = -1;
    int bu = -1;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int e = 0; e < 2; e++) {
                const double w = (a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1]) * (e ? f[2] : 1.0 - f[2]);
                if (!(w > 0.0)) continue;
                const long nidx = ((long)(c[0] + a) * P.n_s + (c[1] + b)) * P.n_t + (c[2] + e);
                const int u = pik[nidx];
                if (u < 0) continue;
                if (w > bw || (w == bw && nidx < bn)) {
                    bw = w;
                    bn = nidx;
                    bu = u;
                }
            }
    return bu;
}

__device__ double interp_f64(const DevInst &P, const float *J, double rv, double rs, double rt)
{
#pragma clang fp contract(off)
    int c[3];
    double f[3];
    cell_of(rv, P.n_v, c[0], f[0]);
    cell_of(rs, P.n_s, c[1], f[1]);
    cell_of(rt, P.n_t, c[2], f[2]);
    double acc = 0.0;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int e = 0; e < 2; e++) {
                const double w = (a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1]) * (e ? f[2] : 1.0 - f[2]);
                if (!(w > 0.0)) continue;
                acc += w * (double)J[((long)(c[0] + a) * P.n_s + (c[1] + b)) * P.n_t + (c[2] + e)];
            }
    return acc;
}

// One instance: x0, the root control u_0*, then at each stage the nearest
// stored control (or the wait at a red signal), exact FP64 dynamics, fuel,
// time and cost accumulated in FP64, terminal cost at N.  The stages depend
// on each other, so one thread runs them.
__device__ void rollout_one(const DevInst &P, const int16_t *__restrict__ pi, const int16_t *__restrict__ u0p,
                            double *__restrict__ traj, int32_t *__restrict__ status)
{
#pragma clang fp contract(off)
    const long S = (long)P.n_v * P.n_s * P.n_t;
    double v = P.v0, xi = P.soc0, t = 0.0, fuel = 0.0, cost = 0.0;
    int st = 0, viol = 0;
    const double nan = __builtin_nan("");
    for (int r = 0; r <= P.N; r++)
        for (int c = 0; c < 8; c++) traj[r * 8 + c] = nan;
    for (int k = 0; k < P.N; k++) {
        double *row = traj + k * 8;
        row[0] = v;
        row[1] = xi;
        row[2] = t;
        row[6] = fuel;
        row[7] = cost;
        int u;
        if (k == 0) {
            u = *u0p;
            if (v > P.vmax[0]) viol++;
        } else {
            const int L = P.light_of_stage[k];
            double tau;
            if (L >= 0 && must_stop(P, L, t, v, tau)) {
                if (v == 0.0 && P.wait) {
                    row[3] = -2.0;
                    t += tau;
                    cost += P.wt * tau;
                    continue;
                }
                viol++;
            }
            if (v > P.vmax[k]) viol++;
            int oog = 0;
            u = policy_lookup(P, pi + (long)k * S, v, xi, t, oog);
            if (oog) viol++;
        }
        if (u < 0) {
            st = -4;
            break;
        }
        const int a = u / P.n_m, b = u % P.n_m;
        row[3] = u;
        row[4] = P.e_lo + a * P.he;
        row[5] = P.m_lo + b * P.hm;
        const PT p = powertrain(P, k, v, a, b);
        double I;
        const bool bok = battery_current(P, p.Pb, xi, I);
        if ((p.st & 4) || !bok) {
            st = -4;
            break;
        }
        if (p.st) viol++;
        fuel += p.mf * p.dt;
        cost += p.cost;
        xi = xi - p.dt * I / P.Cnom;
        v = p.v1;
        t = t + p.dt;
        if (xi < P.s_lo || xi > P.s_hi || t > P.t_f) viol++;
    }
    if (st == 0) {
        double *row = traj + P.N * 8;
        if (v > P.vmax[P.N]) viol++;
        double pen = P.wsoc * (xi - P.xiref) * (xi - P.xiref);
        if (P.terminal_V) {
            double r[3] = {(v - P.v_lo) / P.hv, (xi - P.s_lo) / P.hs, t / P.ht};
            const int n[3] = {P.n_v, P.n_s, P.n_t};
            for (int d = 0; d < 3; d++) r[d] = r[d] < 0.0 ? 0.0 : (r[d] > n[d] - 1 ? n[d] - 1 : r[d]);
            pen += interp_f64(P, P.terminal_V, r[0], r[1], r[2]);
        }
        cost += pen;
        row[0] = v;
        row[1] = xi;
        row[2] = t;
        row[6] = fuel;
        row[7] = cost;
    }
    status[0] = st;
    status[1] = viol;
}

// Every instance of a plan in one launch, one wave per instance (its first
// lane runs the rollout): policy slabs at byte offsets pi_off[b] from pi,
// rows at double offsets traj_off[b] from traj.
__global__ void __launch_bounds__(64) k_rollout_jobs(const DevInst *__restrict__ insts, const char *__restrict__ pi,
                                                     const long long *__restrict__ pi_off,
                                                     const long long *__restrict__ traj_off,
                                                     const int16_t *__restrict__ u0, double *__restrict__ traj,
                                                     int32_t *__restrict__ status)
{
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    rollout_one(insts[b], (const int16_t *)(pi + pi_off[b]), u0 + b, traj + traj_off[b], status + 2 * b);
}

// ------------------------------------------------------------------ adjoint --

struct Cells {
    int c[3];
    double f[3];
};

// Partial derivatives with the control fixed of the stage cost and of the
// three index coordinates of the successor with respect to theta = (M, CdA,
// Crr, w_t, w_soc), from q = v^2 + 2 dd (F_tr - F_road)/M, v1 = sqrt(q),
// dt = 2 dd/(v + v1), SoC shift -dt I/(C_nom h_s), time shift dt/h_t.
__device__ void step_partials(const DevInst &P, double v, const PT &p, double I, double dc[5], double dr[5][3])
{
#pragma clang fp contract(off)
    double dq[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    dq[0] = 2.0 * P.ds * (-P.g * (P.Crr * p.cosa + p.sina) / P.M - (p.Ftr - p.Froad) / (P.M * P.M));
    dq[1] = -P.ds * P.rho * v * v / P.M;
    dq[2] = -2.0 * P.ds * P.g * p.cosa;
    for (int q = 0; q < 5; q++) {
        const double dv1 = p.q > 0.0 ? dq[q] / (2.0 * p.v1) : 0.0;
        const double vs = v + p.v1;
        const double ddt = -2.0 * P.ds / (vs * vs) * dv1;
        dc[q] = (p.mf + P.wt) * ddt + (q == 3 ? p.dt : 0.0);
        dr[q][0] = dv1 / P.hv;
        dr[q][1] = -(I / (P.Cnom * P.hs)) * ddt;
        dr[q][2] = ddt / P.ht;
    }
}

// Derivatives of the trilinear interpolant along each index coordinate inside
// the cell; a coordinate exactly on a grid plane (f = 0 or 1) contributes 0.
__device__ void interp_grad(const DevInst &P, const float *J, const Cells &x, double g[3])
{
#pragma clang fp contract(off)
    // the eight corners, loaded once (cells are at most n - 2 on every axis)
    double Jv[8];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int e = 0; e < 2; e++)
                Jv[(a * 2 + b) * 2 + e] = (double)J[((long)(x.c[0] + a) * P.n_s + (x.c[1] + b)) * P.n_t + (x.c[2] + e)];
    for (int d = 0; d < 3; d++) {
        g[d] = 0.0;
        if (!(x.f[d] > 0.0 && x.f[d] < 1.0)) continue;
        double acc = 0.0;
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                for (int e = 0; e < 2; e++) {
                    const int bits[3] = {a, b, e};
                    double w = 1.0;
                    bool skip = false;
                    for (int o = 0; o < 3; o++) {
                        if (o == d) continue;
                        const double wo = bits[o] ? x.f[o] : 1.0 - x.f[o];
                        if (!(wo > 0.0)) {
                            skip = true;
                            break;
                        }
                        w *= wo;
                    }
                    if (skip) continue;
                    acc += (bits[d] ? 1.0 : -1.0) * w * Jv[(a * 2 + b) * 2 + e];
                }
        g[d] = acc;
    }
}

__device__ void scatter(const DevInst &P, double *rho_next, double r, const Cells &x, bool atomic)
{
#pragma clang fp contract(off)
    for (int a = 0; a < 2; a++) {
        const double wa = a ? x.f[0] : 1.0 - x.f[0];
        if (!(wa > 0.0)) continue;
        for (int b = 0; b < 2; b++) {
            const double wb = b ? x.f[1] : 1.0 - x.f[1];
            if (!(wb > 0.0)) continue;
            for (int e = 0; e < 2; e++) {
                const double we = e ? x.f[2] : 1.0 - x.f[2];
                if (!(we > 0.0)) continue;
                double *dst = rho_next + ((long)(x.c[0] + a) * P.n_s + (x.c[1] + b)) * P.n_t + (x.c[2] + e);
                const double add = r * wa * wb * we;
                if (atomic)
                    unsafeAtomicAdd(dst, add);
                else
                    *dst += add;
            }
        }
    }
}

// Successor cells of a state at speed v, SoC xi with index coordinate rs0 and
// time node m0 under control u; false if the pair is infeasible.
__device__ bool successor_cells(const DevInst &P, int k, double v, double xi, double rs0, int m0, int u, PT &p,
                                double &I, Cells &x)
{
#pragma clang fp contract(off)
    p = powertrain(P, k, v, u / P.n_m, u % P.n_m);
    if (p.st) return false;
    if (!battery_current(P, p.Pb, xi, I)) return false;
    const double rv = (p.v1 - P.v_lo) / P.hv;
    if (!(rv >= 0.0 && rv <= P.n_v - 1)) return false;
    const double rs = rs0 - (p.dt * I) / (P.Cnom * P.hs);
    if (!(rs >= 0.0 && rs <= P.n_s - 1)) return false;
    const double delta = p.dt / P.ht;
    if (!(delta < P.n_t)) return false;
    cell_of(rv, P.n_v, x.c[0], x.f[0]);
    cell_of(rs, P.n_s, x.c[1], x.f[1]);
    const double fl = floor(delta);
    int tc = m0 + (int)fl;
    double ft = delta - fl;
    if (tc > P.n_t - 2) {
        ft += (double)(tc - (P.n_t - 2));
        tc = P.n_t - 2;
        if (ft > 1.0) return false;
    }
    x.c[2] = tc;
    x.f[2] = ft;
    return true;
}

__global__ void k_adj_root(DevInst P, const float *__restrict__ J1, const int16_t *__restrict__ u0p,
                           double *__restrict__ rho1, double *__restrict__ gacc, double *__restrict__ gstage)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int u0 = *u0p;
    const double nan = __builtin_nan("");
    PT p;
    double I;
    Cells x;
    const double rs0 = (P.soc0 - P.s_lo) / P.hs;
    if (u0 < 0 || !successor_cells(P, 0, P.v0, P.soc0, rs0, 0, u0, p, I, x)) {
        for (int q = 0; q < 5; q++) gacc[q] = nan;
        return;
    }
    double dc[5], dr[5][3], gJ[3];
    step_partials(P, P.v0, p, I, dc, dr);
    interp_grad(P, J1, x, gJ);
    for (int q = 0; q < 5; q++) gacc[q] += dc[q] + dr[q][0] * gJ[0] + dr[q][1] * gJ[1] + dr[q][2] * gJ[2];
    // stage 0's share of dV/dC_rr (slot 0 of stage 0; the other slots stay 0)
    if (gstage) gstage[0] = dc[2] + dr[2][0] * gJ[0] + dr[2][1] * gJ[1] + dr[2][2] * gJ[2];
    scatter(P, rho1, 1.0, x, false);
}

// Workgroups of the adjoint kernels (each owns a slot of partial gradient
// sums, so no two workgroups add into the same memory).
constexpr int kAdjBlocks = 1024;

// Sum g over the workgroup (wave shuffles, then one LDS step) and add it to
// the workgroup's own slot gpart[blockIdx.x][0..4]; with gcrr, also store
// this launch's C_rr sum (component 2) in gcrr[blockIdx.x].
__device__ inline void block_add5(double g[5], double *gpart, double *gcrr = nullptr)
{
    __shared__ double red[16][5];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    for (int q = 0; q < 5; q++) {
        double x = g[q];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) red[w][q] = x;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double x = 0.0;
        for (int ww = 0; ww < nw; ww++) x += red[ww][threadIdx.x];
        // the workgroup's own slot, one launch at a time: an add without a
        // returned value, so the workgroup does not wait on a read of it
        unsafeAtomicAdd(&gpart[(long)blockIdx.x * 5 + threadIdx.x], x);
        if (gcrr && threadIdx.x == 2) gcrr[blockIdx.x] = x;
    }
}

// The workgroup's sums of a and b into slot[2 blockIdx.x + 0, 1].
__device__ inline void block_store2(double a, double b, double *slot)
{
    __shared__ double red2[16][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    if (lane == 0) {
        red2[w][0] = a;
        red2[w][1] = b;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double x = 0.0;
        for (int ww = 0; ww < nw; ww++) x += red2[ww][threadIdx.x];
        slot[(long)blockIdx.x * 2 + threadIdx.x] = x;
    }
}

// dV/dO, dV/dR and dV/dC of every signal L from the kAdjBlocks slot pairs of
// its stage: offset and red time move the wait alike, the cycle by n whole
// cycles per node (the red masks are constant between switching instants).
__global__ void __launch_bounds__(64) k_adj_spat(int n_lights, const double *__restrict__ gspat,
                                                 const double *__restrict__ grad, double *__restrict__ dspat)
{
#pragma clang fp contract(off)
    const bool none = grad[0] != grad[0];   // x0 had no admissible control: not a number, like grad
    for (int L = blockIdx.x * blockDim.x + threadIdx.x; L < n_lights; L += gridDim.x * blockDim.x) {
        double o = 0.0, c = 0.0;
        for (int b = 0; b < kAdjBlocks; b++) {
            o += gspat[((long)L * kAdjBlocks + b) * 2];
            c += gspat[((long)L * kAdjBlocks + b) * 2 + 1];
        }
        dspat[3 * L + 0] = none ? grad[0] : o;
        dspat[3 * L + 1] = none ? grad[0] : o;
        dspat[3 * L + 2] = none ? grad[0] : c;
    }
}

// dV/dG_k for every step k: the grade of step k enters only the road load,
// like C_rr, with dF_road/dG = M g cos^3 a (1 - C_rr G) against dF_road/dC_rr
// = M g cos a, so dV/dG_k is cos a (cos a - C_rr sin a) times step k's share
// of dV/dC_rr (summed over the kAdjBlocks slots of gstage[k]).
__global__ void __launch_bounds__(256) k_adj_grade(DevInst P, const double *__restrict__ gstage,
                                                   const double *__restrict__ grad, double *__restrict__ dgrade)
{
#pragma clang fp contract(off)
    const bool none = grad[0] != grad[0];   // x0 had no admissible control: not a number, like grad
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < P.N; k += gridDim.x * blockDim.x) {
        double x = 0.0;
        for (int b = 0; b < kAdjBlocks; b++) x += gstage[(long)k * kAdjBlocks + b];
        dgrade[k] = none ? grad[0] : P.cosa[k] * (P.cosa[k] - P.Crr * P.sina[k]) * x;
    }
}

// grad[q] += sum over the kAdjBlocks slots of component q.
__global__ void __launch_bounds__(256) k_adj_reduce(const double *__restrict__ gpart, double *__restrict__ grad)
{
    __shared__ double red[4][5];
    double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < kAdjBlocks; b += blockDim.x)
        for (int q = 0; q < 5; q++) g[q] += gpart[(long)b * 5 + q];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q = 0; q < 5; q++) {
        double x = g[q];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) red[w][q] = x;
    }
    __syncthreads();
    if (threadIdx.x < 5) grad[threadIdx.x] += red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                                               red[3][threadIdx.x];
}

// The FP64 step terms of one stage that depend on the speed node and the
// control only (Eq. 5a, 2, 1 and their theta partials, as step_partials): a
// table over (i, u), so that an occupied node only adds the battery and SoC
// terms.  ok = 0 for a pair the stage does not admit (the node's successor
// is then not formed).
struct AdjEntry {
    double dt, Pb, fv, ft;
    double dc[3];        // d cost / d(M, CdA, Crr)
    double drv[3];       // d r_v / d(M, CdA, Crr)
    double ddt[3];       // d dt / d(M, CdA, Crr)
    double drt[3];       // d r_t / d(M, CdA, Crr)
    int cv, dtc, ok, pad;
};

__global__ void __launch_bounds__(256) k_adj_table(DevInst P, int k, AdjEntry *__restrict__ tab)
{
#pragma clang fp contract(off)
    const long n = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (n >= (long)P.n_v * P.n_u) return;
    const int i = (int)(n / P.n_u), u = (int)(n % P.n_u);
    const double v = P.v_lo + i * P.hv;
    const PT p = powertrain(P, k, v, u / P.n_m, u % P.n_m);
    AdjEntry e;
    e.ok = 0;
    e.dt = p.dt;
    e.Pb = p.Pb;
    e.cv = 0;
    e.fv = 0.0;
    e.dtc = 0;
    e.ft = 0.0;
    const double rv = (p.v1 - P.v_lo) / P.hv;
    const double delta = p.dt / P.ht;
    if (p.st == 0 && rv >= 0.0 && rv <= P.n_v - 1 && delta < P.n_t) {
        e.ok = 1;
        cell_of(rv, P.n_v, e.cv, e.fv);
        const double fl = floor(delta);
        e.dtc = (int)fl;
        e.ft = delta - fl;
    }
    // the partials of step_partials for theta = M, CdA, Crr (w_t enters the
    // cost as dt, w_soc only the terminal cost)
    double dq[3];
    dq[0] = 2.0 * P.ds * (-P.g * (P.Crr * p.cosa + p.sina) / P.M - (p.Ftr - p.Froad) / (P.M * P.M));
    dq[1] = -P.ds * P.rho * v * v / P.M;
    dq[2] = -2.0 * P.ds * P.g * p.cosa;
    for (int q = 0; q < 3; q++) {
        const double dv1 = p.q > 0.0 ? dq[q] / (2.0 * p.v1) : 0.0;
        const double vs = v + p.v1;
        const double ddt = -2.0 * P.ds / (vs * vs) * dv1;
        e.dc[q] = (p.mf + P.wt) * ddt;
        e.drv[q] = dv1 / P.hv;
        e.ddt[q] = ddt;
        e.drt[q] = ddt / P.ht;
    }
    e.pad = 0;
    tab[n] = e;
}

// Stage k >= 1: every node with occupancy rho > 0 follows its stored control:
// gradient terms weighted by rho, and rho times the interpolation weights
// added to the stage k+1 occupancy.  Wait nodes add rho * tau to dV/dw_t and
// move in time only.  Nodes without a control keep J_inf and stop the mass.
// Each workgroup takes a chunk of CHUNK consecutive nodes, gathers the
// ones with rho > 0 (and their rho) into LDS lists, zeroing them in rho (so
// that the buffer is all zero again when it becomes the occupancy two stages
// later), and then runs the FP64 work on full waves: per node the (i, u)
// entry of the stage table, the battery current and SoC cell (Eq. 5b), the
// interpolation gradient and the scatter.
constexpr int kAdjThreads = 256;

// SPAT: also the signal-timing sums of the wait nodes (a separate instance, so
// that the plain adjoint keeps its registers).  CHUNK: 1024 nodes, or 2048 on
// grids with at least two such chunks per workgroup (more SoC-row neighbours
// in one chunk, at four workgroups per CU instead of five).
template <bool SPAT, int CHUNK>
__global__ void __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(CHUNK > 1024 ? 4 : 5, 8)))
k_adj_stage(DevInst P, int k, const float *__restrict__ Jn, const int16_t *__restrict__ pik,
            const TLEntry *__restrict__ tl, const AdjEntry *__restrict__ tab, double *__restrict__ rho,
            double *__restrict__ rho_next, double *__restrict__ gacc, double *__restrict__ gcrr,
            double *__restrict__ gspat)
{
#pragma clang fp contract(off)
    __shared__ short s_list[CHUNK];              // list slot -> chunk position
    __shared__ double s_rho[CHUNK];
    __shared__ short s_slot[CHUNK];              // chunk position -> list slot, -1 if unoccupied
    __shared__ short s_u[CHUNK];                 // list slot -> stored control
    __shared__ int s_key[3][kAdjThreads];        // per slot of the pass: successor speed, SoC, time cell
    __shared__ double s_up[4][kAdjThreads];      // per slot of the pass: its upper-SoC terms
    __shared__ int s_cnt;
    double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double sO = 0.0, sC = 0.0;   // signal timing: sum of rho dval/dtau, and of rho n dval/dtau
    const long S = (long)P.n_v * P.n_s * P.n_t;
    const int lane = threadIdx.x & 63;
    for (long c0 = blockIdx.x * (long)CHUNK; c0 < S; c0 += (long)gridDim.x * CHUNK) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        // all loads of the chunk's occupancy in flight at once, then the
        // controls of the occupied nodes
        constexpr int kPer = CHUNK / kAdjThreads;
        double rv[kPer];
        for (int q = 0; q < kPer; q++) {
            const long n = c0 + q * kAdjThreads + threadIdx.x;
            rv[q] = n < S ? rho[n] : 0.0;
        }
        int16_t uv[kPer];
        for (int q = 0; q < kPer; q++) uv[q] = rv[q] > 0.0 ? pik[c0 + q * kAdjThreads + threadIdx.x] : (int16_t)-1;
        for (int q = 0; q < kPer; q++) {
            const int jj = q * kAdjThreads + (int)threadIdx.x;
            const bool act = rv[q] > 0.0;
            const unsigned long long msk = __ballot(act);
            int off = 0;
            if (lane == 0 && msk) off = atomicAdd(&s_cnt, __popcll(msk));
            off = __shfl(off, 0);
            s_slot[jj] = -1;
            if (act) {
                const int slot = off + __popcll(msk & ((1ull << lane) - 1ull));
                s_list[slot] = (short)jj;
                s_rho[slot] = rv[q];
                s_u[slot] = uv[q];
                s_slot[jj] = (short)slot;
                rho[c0 + jj] = 0.0;
            }
        }
        __syncthreads();
        const int na = s_cnt;
        // Waves walk the list together (every lane takes part in the
        // exchanges below, past the list's end too), a pass of kAdjThreads
        // list slots at a time.  Occupied nodes come in node order, so
        // neighbouring lanes often hold nodes m - 1 and m of one (speed, SoC)
        // row under the same control, and the slot of the node one SoC row
        // down is usually in the same pass: their successors then share
        // corner cells.  Terms that go to one cell are added up first and
        // sent with one atomic (time neighbours through shuffles, SoC
        // neighbours through LDS).
        for (int a0 = 0; a0 < na; a0 += blockDim.x) {
            const int a = a0 + (int)threadIdx.x;
            const bool live = a < na;
            const int jj = live ? s_list[a] : 0;
            const long n = c0 + jj;
            const double r = live ? s_rho[a] : 0.0;
            const int m = (int)(n % P.n_t);
            const long ij = n / P.n_t;
            const int j = (int)(ij % P.n_s);
            const int i = (int)(ij / P.n_s);
            const int u = live ? (int)s_u[a] : -1;
            bool scat = false;     // a regular successor whose 8 corners this lane scatters
            Cells x;
            x.c[0] = x.c[1] = x.c[2] = 0;
            x.f[0] = x.f[1] = x.f[2] = 0.0;
            if (u == -2) {
                const TLEntry e = tl[m];
                g[3] += r * e.tau;
                const long base = ((long)i * P.n_s + j) * P.n_t;
                if (SPAT) {
                    // the wait value w_t tau + J_{k+1}(t_m + tau) moves with
                    // tau = R - phase, phase = t - O - n C: dtau/dO = dtau/dR
                    // = 1, dtau/dC = n (Eq. 5c, 8); the time derivative of the
                    // lerp counts only strictly inside a cell
                    double gt = 0.0;
                    if (e.wf > 0.0 && e.wf < 1.0) gt = (double)Jn[base + e.wc + 1] - (double)Jn[base + e.wc];
                    const double dval = P.wt + gt / P.ht;
                    sO += r * dval;
                    sC += r * dval * (double)e.ncyc;
                }
                if (1.0 - e.wf > 0.0) unsafeAtomicAdd(&rho_next[base + e.wc], r * (1.0 - e.wf));
                if (e.wf > 0.0) unsafeAtomicAdd(&rho_next[base + e.wc + 1], r * e.wf);
            } else if (u >= 0) {
                // the successor exactly as successor_cells forms it, the
                // (i, u) terms from the stage table
                const AdjEntry &e = tab[(long)i * P.n_u + u];
                const double xi = P.s_lo + j * P.hs;
                double I = 0.0;
                double rs = -1.0;
                if (e.ok && battery_current(P, e.Pb, xi, I)) rs = (double)j - (e.dt * I) / (P.Cnom * P.hs);
                if (rs >= 0.0 && rs <= P.n_s - 1) {
                    x.c[0] = e.cv;
                    x.f[0] = e.fv;
                    cell_of(rs, P.n_s, x.c[1], x.f[1]);
                    int tc = m + e.dtc;
                    double ft = e.ft;
                    if (tc > P.n_t - 2) {
                        ft += (double)(tc - (P.n_t - 2));
                        tc = P.n_t - 2;
                    }
                    x.c[2] = tc;
                    x.f[2] = ft;
                    if (ft <= 1.0) {
                        scat = true;
                        double gJ[3];
                        interp_grad(P, Jn, x, gJ);
                        const double sI = -(I / (P.Cnom * P.hs));
                        for (int q = 0; q < 3; q++)
                            g[q] += r * (e.dc[q] + e.drv[q] * gJ[0] + (sI * e.ddt[q]) * gJ[1] + e.drt[q] * gJ[2]);
                        g[3] += r * e.dt;
                    }
                }
            }
            // the eight terms t[(ca * 2 + cb) * 2 + ce] for speed, SoC and time
            // corners ca, cb, ce of the successor cell (0 where a weight is 0)
            double t[8];
            for (int q = 0; q < 8; q++) {
                const int ca = q >> 2, cb = (q >> 1) & 1, ce = q & 1;
                const double wa = ca ? x.f[0] : 1.0 - x.f[0];
                const double wb = cb ? x.f[1] : 1.0 - x.f[1];
                const double we = ce ? x.f[2] : 1.0 - x.f[2];
                t[q] = scat && wa > 0.0 && wb > 0.0 && we > 0.0 ? r * wa * wb * we : 0.0;
            }
            const int kcv = scat ? x.c[0] : -1;
            // time merge: the previous lane's successor lies one time cell
            // below this one in the same speed and SoC cells (its upper time
            // corners are this lane's lower ones)
            {
                const int p_cv = __shfl_up(kcv, 1);
                const int p_cs = __shfl_up(x.c[1], 1);
                const int p_tc = __shfl_up(x.c[2], 1);
                double p_up[4];
                for (int q = 0; q < 4; q++) p_up[q] = __shfl_up(t[q * 2 + 1], 1);
                const bool merge = scat && lane > 0 && p_cv == kcv && p_cs == x.c[1] && p_tc == x.c[2] - 1;
                const bool absorbed = __shfl_down((int)merge, 1) && lane < 63;
                for (int q = 0; q < 4; q++) {
                    if (merge) t[q * 2] += p_up[q];
                    if (absorbed) t[q * 2 + 1] = 0.0;
                }
            }
            // SoC merge through LDS, between slots of this pass: the node one
            // SoC row down, if its successor lies one SoC cell below this one
            // in the same speed and time cells, sends its upper-SoC terms
            const int sl = a - a0;
            if (live) {
                s_key[0][sl] = kcv;
                s_key[1][sl] = x.c[1];
                s_key[2][sl] = x.c[2];
                for (int ca = 0; ca < 2; ca++)
                    for (int ce = 0; ce < 2; ce++) s_up[ca * 2 + ce][sl] = t[(ca * 2 + 1) * 2 + ce];
            }
            __syncthreads();
            if (scat) {
                const int pp = jj - P.n_t, pn = jj + P.n_t;
                const int sp = pp >= 0 ? (int)s_slot[pp] - a0 : -1;
                const int ss = pn < CHUNK ? (int)s_slot[pn] - a0 : -1;
                const bool take = sp >= 0 && sp < kAdjThreads && s_key[0][sp] == kcv && s_key[1][sp] == x.c[1] - 1 &&
                                  s_key[2][sp] == x.c[2];
                const bool give = ss >= 0 && ss < kAdjThreads && s_key[0][ss] == kcv && s_key[1][ss] == x.c[1] + 1 &&
                                  s_key[2][ss] == x.c[2];
                for (int q = 0; q < 8; q++) {
                    const int ca = q >> 2, cb = (q >> 1) & 1, ce = q & 1;
                    double v = t[q];
                    if (cb == 0 && take) v += s_up[ca * 2 + ce][sp];
                    if (cb == 1 && give) v = 0.0;
                    if (v > 0.0)
                        unsafeAtomicAdd(
                            rho_next + ((long)(x.c[0] + ca) * P.n_s + (x.c[1] + cb)) * P.n_t + (x.c[2] + ce), v);
                }
            }
            __syncthreads();   // the pass's keys are read before the next pass rewrites them
        }
        __syncthreads();   // the list is read before the next chunk rewrites it
    }
    block_add5(g, gacc, gcrr);
    if (SPAT) block_store2(sO, sC, gspat);
}

// Stage N: dV/dw_soc gains rho_N (xi - xi_ref)^2 on nodes below J_inf.
__global__ void __launch_bounds__(256) k_adj_terminal(DevInst P, const float *__restrict__ JN,
                                                      const double *__restrict__ rho, double *__restrict__ gacc)
{
#pragma clang fp contract(off)
    double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const long S = (long)P.n_v * P.n_s * P.n_t;
    const float Jinf = (float)P.Jinf;
    for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < S; n += (long)gridDim.x * blockDim.x) {
        const double r = rho[n];
        if (!(r > 0.0) || !(JN[n] < Jinf)) continue;
        const int j = (int)((n / P.n_t) % P.n_s);
        const double d = P.s_lo + j * P.hs - P.xiref;
        g[4] += r * d * d;
    }
    block_add5(g, gacc);
}

__global__ void k_fill_f64(double *p, long n, double v)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) p[q] = v;
}

static int grid_for(long n)
{
    long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

int launch_rollout_jobs(const DevInst *insts, int n_inst, const void *pi, const long long *pi_off,
                        const long long *traj_off, const int16_t *u0, double *traj, int32_t *status, hipStream_t s)
{
    hipLaunchKernelGGL(k_rollout_jobs, dim3(n_inst), dim3(64), 0, s, insts, (const char *)pi, pi_off, traj_off, u0, traj,
                       status);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}


int launch_fill_f64(double *p, long n, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_adjoint_reduce(const double *gpart, double *grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(256), 0, s, gpart, grad);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_adjoint_root(const DevInst &P, const float *J1, const int16_t *u0, double *rho1, double *gacc,
                        double *gstage, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_root, dim3(1), dim3(64), 0, s, P, J1, u0, rho1, gacc, gstage);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

size_t adjoint_table_bytes(const DevInst &P) { return sizeof(AdjEntry) * (size_t)P.n_v * P.n_u; }

int launch_adjoint_table(const DevInst &P, int k, void *tab, hipStream_t s)
{
    const long n = (long)P.n_v * P.n_u;
    hipLaunchKernelGGL(k_adj_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, k, (AdjEntry *)tab);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_adjoint_stage(const DevInst &P, int k, const float *Jn, const int16_t *pik, const TLEntry *tl,
                         const void *tab, double *rho, double *rho_next, double *gacc, double *gstage,
                         double *gspat_L, bool force_wide, hipStream_t s)
{
    // kAdjBlocks workgroups walk the chunks, each adding into its own slot
    // (and, at a signal, storing its pair of gspat_L)
    double *gcrr = gstage ? gstage + (long)k * kAdjBlocks : nullptr;
    const AdjEntry *t = (const AdjEntry *)tab;
    const long S = (long)P.n_v * P.n_s * P.n_t;
    const bool wide = force_wide || S >= 2L * 2048 * kAdjBlocks;
    const dim3 g(kAdjBlocks), b(kAdjThreads);
    if (tl && gspat_L) {
        if (wide)
            hipLaunchKernelGGL((k_adj_stage<true, 2048>), g, b, 0, s, P, k, Jn, pik, tl, t, rho, rho_next, gacc, gcrr,
                               gspat_L);
        else
            hipLaunchKernelGGL((k_adj_stage<true, 1024>), g, b, 0, s, P, k, Jn, pik, tl, t, rho, rho_next, gacc, gcrr,
                               gspat_L);
    } else {
        if (wide)
            hipLaunchKernelGGL((k_adj_stage<false, 2048>), g, b, 0, s, P, k, Jn, pik, tl, t, rho, rho_next, gacc, gcrr,
                               nullptr);
        else
            hipLaunchKernelGGL((k_adj_stage<false, 1024>), g, b, 0, s, P, k, Jn, pik, tl, t, rho, rho_next, gacc, gcrr,
                               nullptr);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_adjoint_spat(int n_lights, const double *gspat, const double *grad, double *dspat, hipStream_t s)
{
    if (n_lights <= 0) return 0;
    hipLaunchKernelGGL(k_adj_spat, dim3((n_lights + 63) / 64), dim3(64), 0, s, n_lights, gspat, grad, dspat);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_adjoint_terminal(const DevInst &P, const float *JN, const double *rho, double *gacc, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_terminal, dim3(kAdjBlocks), dim3(256), 0, s, P, JN, rho, gacc);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_adjoint_grade(const DevInst &P, const double *gstage, const double *grad, double *dgrade, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_grade, dim3((P.N + 255) / 256), dim3(256), 0, s, P, gstage, grad, dgrade);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

size_t adjoint_grade_slots() { return (size_t)kAdjBlocks; }

}  // namespace ecodp
