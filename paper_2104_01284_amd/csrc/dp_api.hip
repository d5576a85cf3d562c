// Host side of the ecodp C ABI: validation, FP64 host preprocessing (grade
// trigonometry, speed limits, signal red masks and wait times, Eq. 5c / 8),
// buffer layout, and the enqueueing of the kernels on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ecodp.h"
#include "dp_internal.h"

using namespace ecodp;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(DP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Set while build_window_plan builds a closed loop's window plan: every stage
// builds its own tables, and the SoC-shift bound is at least h_min.
struct WindowBuild {
    bool on = false;
    int h_min = 0;
};
thread_local WindowBuild t_window;

struct Inst {
    DevInst P;                 // device pointers filled at build
    int N = 0;
    size_t S = 0;              // slab elements
    std::vector<int> light_of_stage;
    int n_lights = 0;
    size_t J_off = 0, pi_off = 0, traj_off = 0;
    size_t scr_st = 0, scr_bat = 0, scr_rho = 0, scr_nf = 0, scr_pw = 0;
    int sweep = 0;             // 1 = simple per-node kernel, 2 = grouped LDS kernel
    int jt = 8;                // SoC rows per workgroup of the grouped kernel
    int nsplit = 1;            // largest number of control slices of any of its stages
    int split_opt = 0;         // caller's control slices (0 = chosen per round)
    int wg_opt = 0;            // caller's resident sweep workgroups per CU (0 = by LDS)
    size_t scr_pv = 0, scr_pu = 0, scr_rec = 0;
    size_t tab_stride = 0;     // bytes from the first stage-table set to the second (grouped sweep)
    int grid = 0;              // persistent workgroups of a grouped sweep of this instance alone
    int H = 0;                 // bound on the SoC-cell shift of one step
    size_t tl_dev_off = 0;     // offset (entries) of this instance's TL table in the plan's TL array
    int64_t evals = 0;
    std::vector<int> job_of_k; // grouped sweep: index of the (instance, k) job in the plan's job table
    std::vector<double> l_cycle, l_red, l_off, l_yel;   // signals, kept for dp_set_state
    std::vector<char> same_tables;               // [k]: stage k's tables equal stage k+1's
};

// One grouped-sweep launch of a round: the jobs of one (tile, pitch, block)
// class, largest work per item first.
struct SweepLaunch {
    int jt = 0, pitch = 0, threads = 0;
    int job_begin = 0, njobs = 0, items = 0, grid = 0;
    size_t lds = 0;
    size_t ib_off = 0;         // first entry of the launch's item_begin table
    int q_slot = 0;            // queue counters
    double work = 0.0;         // estimated lane-steps, for ordering the launches of a round
};

// Round r of a solve holds stage N_b - 1 - r of every instance b with N_b > r.
struct Round {
    int job_begin = 0, njobs = 0;      // grouped-sweep jobs, ordered by launch
    int max_nv = 0;
    long max_records = 0, max_nodes = 0;
    // jobs whose stage tables differ from their instance's previous stage
    // (the others reuse the table set of the previous round)
    int bjob_begin = 0, nbjobs = 0, bmax_nv = 0;
    long bmax_records = 0;
    bool any_split = false;
    std::vector<SweepLaunch> sweeps;
    std::vector<int> simple;           // instances on the simple per-node sweep
};

}  // namespace

struct dp_plan {
    int device = 0;
    int n_cu = 256, lds_per_cu = 160 * 1024;
    uint32_t flags = 0;
    dp_options opt{};
    std::vector<Inst> inst;
    size_t bytes_J = 0, bytes_pi = 0, bytes_scratch = 0;
    void *dev_params = nullptr;      // all per-instance device arrays, one allocation
    TLEntry *dev_tl = nullptr;
    bool solved = false;
    std::vector<hipEvent_t> ev;      // DP_TIMING: begin/end pairs of sweep launches
    int n_ev_used = 0;
    // grouped sweep tables: parameter blocks, jobs, per-launch item offsets
    std::vector<StageJob> jobs;
    std::vector<StageJob> bjobs;     // per round, the jobs that build stage tables
    StageJob *dev_bjobs = nullptr;
    long long *dev_roll = nullptr;   // per instance [4][n_inst]: pi byte offset, traj double offset,
                                     // J_1 and J_N byte offsets
    long max_slab = 0;               // largest slab of any instance
    std::vector<Round> rounds;
    // persistent batched sweep (several instances, DP_ROUNDS unset): one
    // launch per kernel class over every stage, tables of every distinct
    // stage built before it
    struct PClass {
        int jt = 0, pitch = 0, threads = 0, grid = 0;
        size_t lds = 0;
        int xjb_off = 0;             // ints into dev_pint: job bounds [n_xcd + 1], item totals [n_xcd]
        int claim_off = 0;           // ints from scr_pc: claim counters [n_xcd]
        double work = 0.0;
        std::vector<int> members;
    };
    bool persist = false;
    int n_xcd = 8;
    std::vector<PClass> pclasses;
    void *dev_ptables = nullptr;     // PJob queues, their bounds and the table-build jobs
    PJob *dev_pjobs = nullptr;
    int *dev_pint = nullptr;
    StageJob *dev_pbjobs = nullptr;
    int n_pbjobs = 0, pb_max_nv = 0;
    long pb_max_records = 0;
    size_t scr_pc = 0;               // persistent counters: claims of every class, then done per instance
    long n_pc = 0;
    int done_off = 0;
    long long spin_limit = 1LL << 22;   // polls of a persistent wait (each a load and a short sleep): seconds
    void *dev_tables = nullptr;
    DevInst *dev_insts = nullptr;
    StageJob *dev_jobs = nullptr;
    int *dev_ib = nullptr;
    int *dev_err = nullptr;                  // device error word (kDevErr* bits), sticky until read
    unsigned long long *dev_count = nullptr; // per instance: evaluations executed since the last solve began
    size_t scr_q = 0;                // 8 queue counters per sweep launch, then 8 for dp_stage
    size_t scr_gpart = 0;            // adjoint partial gradient sums
    size_t scr_gstage = 0;           // adjoint per-stage C_rr shares (grade sensitivities)
    size_t scr_gspat = 0;            // adjoint per-signal wait sums (signal-timing sensitivities)
    size_t scr_adjtab = 0;           // adjoint per-(speed node, control) table of one stage
    int n_q_slots = 0;
    // independent sweep launches of a round run on these streams side by side
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[kSide] = {nullptr, nullptr, nullptr};
    // the stage tables of the next round are built on this stream
    hipStream_t tstream = nullptr;
    hipEvent_t tfork = nullptr, tjoin = nullptr;
    // dp_set_state: pinned staging of the moved parameter block and signal
    // tables, reused once the previous upload has been consumed
    void *state_host = nullptr;
    size_t state_bytes = 0;
    hipEvent_t state_ev = nullptr;
    bool state_pending = false;
    // DP_GRAPH: the captured solve and the buffers it was captured with
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const void *graph_key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace {

bool finite(double x) { return std::isfinite(x); }

int validate(const dp_problem_desc &d, int b)
{
    if (d.n_stages < 1 || d.n_stages > 100000) return fail(DP_EINVAL, "instance %d: n_stages %d out of range", b, d.n_stages);
    if (!(finite(d.ds) && d.ds > 0)) return fail(DP_EINVAL, "instance %d: ds must be finite and > 0", b);
    if (!d.grade) return fail(DP_EINVAL, "instance %d: grade is NULL", b);
    for (int k = 0; k < d.n_stages; k++)
        if (!finite(d.grade[k])) return fail(DP_EINVAL, "instance %d: grade[%d] not finite", b, k);
    if (d.v_max)
        for (int k = 0; k <= d.n_stages; k++)
            if (!(finite(d.v_max[k]) && d.v_max[k] >= 0)) return fail(DP_EINVAL, "instance %d: v_max[%d] invalid", b, k);
    if (d.n_lights < 0) return fail(DP_EINVAL, "instance %d: n_lights < 0", b);
    if (d.n_lights > 0 && !(d.light_stage && d.light_cycle && d.light_red && d.light_offset))
        return fail(DP_EINVAL, "instance %d: light arrays are NULL", b);
    for (int L = 0; L < d.n_lights; L++) {
        const int k = d.light_stage[L];
        if (k < 1 || k > d.n_stages - 1) return fail(DP_EINVAL, "instance %d: light %d at stage %d not in [1, N-1]", b, L, k);
        for (int L2 = 0; L2 < L; L2++)
            if (d.light_stage[L2] == k) return fail(DP_EINVAL, "instance %d: two lights at stage %d", b, k);
        if (!(finite(d.light_cycle[L]) && d.light_cycle[L] > 0)) return fail(DP_EINVAL, "instance %d: light %d cycle invalid", b, L);
        if (!(finite(d.light_red[L]) && d.light_red[L] > 0 && d.light_red[L] <= d.light_cycle[L]))
            return fail(DP_EINVAL, "instance %d: light %d red invalid", b, L);
        if (!finite(d.light_offset[L])) return fail(DP_EINVAL, "instance %d: light %d offset invalid", b, L);
        if (d.light_yellow) {
            const double Y = d.light_yellow[L];
            if (!(finite(Y) && Y >= 0 && Y <= d.light_cycle[L] - d.light_red[L]))
                return fail(DP_EINVAL, "instance %d: light %d yellow invalid (0 <= Y <= C - R)", b, L);
            if (Y > 0 && !(d.konst[10] < 0))
                return fail(DP_EINVAL, "instance %d: a yellow phase needs a braking limit a_min < 0", b);
        }
    }
    if (!(finite(d.t0_abs) && finite(d.v0) && finite(d.soc0))) return fail(DP_EINVAL, "instance %d: x0 not finite", b);
    if (!(finite(d.v_lo) && finite(d.v_hi) && d.v_lo >= 0 && d.v_hi > d.v_lo && d.n_v >= 2))
        return fail(DP_EINVAL, "instance %d: speed grid invalid", b);
    if (!(finite(d.soc_lo) && finite(d.soc_hi) && d.soc_hi > d.soc_lo && d.n_soc >= 2))
        return fail(DP_EINVAL, "instance %d: SoC grid invalid", b);
    if (!(finite(d.t_f) && d.t_f > 0 && d.n_t >= 2)) return fail(DP_EINVAL, "instance %d: time grid invalid", b);
    if (!(finite(d.te_lo) && finite(d.te_hi) && d.te_hi >= d.te_lo && d.n_te >= 1 && (d.n_te > 1 || d.te_hi == d.te_lo)))
        return fail(DP_EINVAL, "instance %d: engine torque grid invalid", b);
    if (!(finite(d.tm_lo) && finite(d.tm_hi) && d.tm_hi >= d.tm_lo && d.n_tm >= 1 && (d.n_tm > 1 || d.tm_hi == d.tm_lo)))
        return fail(DP_EINVAL, "instance %d: motor torque grid invalid", b);
    if (!(d.v0 >= 0 && d.soc0 >= d.soc_lo && d.soc0 <= d.soc_hi)) return fail(DP_EINVAL, "instance %d: x0 outside the grid", b);
    for (int q = 0; q < 5; q++)
        if (!finite(d.theta[q])) return fail(DP_EINVAL, "instance %d: theta[%d] not finite", b, q);
    if (!(d.theta[0] > 0 && d.theta[1] >= 0 && d.theta[2] >= 0 && d.theta[3] >= 0 && d.theta[4] >= 0))
        return fail(DP_EINVAL, "instance %d: theta out of range", b);
    for (int q = 0; q < 16; q++)
        if (!finite(d.konst[q])) return fail(DP_EINVAL, "instance %d: konst[%d] not finite", b, q);
    const double *K = d.konst;
    if (!(K[2] > 0 && K[3] > 0 && K[4] > 0 && K[5] > 0 && K[6] > 0 && K[9] > 0 && K[13] > 0 && K[10] < K[11] &&
          K[14] >= 0 && K[15] >= 0))
        return fail(DP_EINVAL, "instance %d: vehicle constants out of range", b);
    for (int q = 0; q < 6; q++)
        if (!finite(d.fuel[q])) return fail(DP_EINVAL, "instance %d: fuel[%d] not finite", b, q);
    if ((long)d.n_te * d.n_tm > 32767) return fail(DP_EUNSUPPORTED, "instance %d: more than 32767 controls", b);
    if (d.n_v > 32767 || d.n_soc > 32767) return fail(DP_EUNSUPPORTED, "instance %d: grid too large", b);
    if (d.n_t > 1024) return fail(DP_EUNSUPPORTED, "instance %d: n_t > 1024", b);
    if ((long)d.n_v * d.n_soc * d.n_t > (1L << 30))
        return fail(DP_EUNSUPPORTED, "instance %d: more than 2^30 states per stage (grid too large)", b);
    if (d.flags & ~(DP_WAIT_AT_RED | DP_TERMINAL_DEVICE)) return fail(DP_EINVAL, "instance %d: unknown flags", b);
    if (d.flags & DP_TERMINAL_DEVICE) {
        if (!d.terminal_V) return fail(DP_EINVAL, "instance %d: DP_TERMINAL_DEVICE without terminal_V", b);
        hipPointerAttribute_t a;
        if (hipPointerGetAttributes(&a, d.terminal_V) != hipSuccess ||
            (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)) {
            (void)hipGetLastError();
            return fail(DP_EINVAL, "instance %d: DP_TERMINAL_DEVICE but terminal_V is not device memory", b);
        }
    } else if (d.terminal_V) {
        // costs are non-negative (the sweep's minimum relies on it); a NaN
        // terminal value makes the node J_inf
        const long S = (long)d.n_v * d.n_soc * d.n_t;
        for (long n = 0; n < S; n++)
            if (d.terminal_V[n] < 0.0f)
                return fail(DP_EINVAL, "instance %d: terminal_V[%ld] = %g is negative", b, n, (double)d.terminal_V[n]);
    }
    return DP_OK;
}

double gstep(double lo, double hi, int n) { return n > 1 ? (hi - lo) / (n - 1) : 0.0; }

// Signal table of one light over the time grid [0, t_f] x n_t (Eq. 5c, 8):
// per time node the red flag and, for a stopped vehicle, the wait to the end
// of red in index space; FP64 on the host.
void build_tl(double C, double R, double O, double Y, double t0_abs, double t_f, int n_t, double wt, TLEntry *out)
{
    const double ht = gstep(0.0, t_f, n_t);
    for (int m = 0; m < n_t; m++) {
        TLEntry e;
        std::memset(&e, 0, sizeof e);
        const double tm = 0.0 + m * ht;
        double ph = std::fmod(t0_abs + tm - O, C);
        if (ph < 0.0) ph += C;
        e.red = ph < R ? 1 : 0;
        // yellow: the Y seconds before red (Sec. III)
        e.yel = !e.red && Y > 0.0 && ph >= C - Y ? 1 : 0;
        e.ys = e.yel ? ph - (C - Y) : 0.0;
        e.wc = -1;
        // a vehicle at rest has to stop in red, and in yellow once it has
        // begun (tl_stop at v = 0); it waits until green
        if (e.red || (e.yel && e.ys > 0.0)) {
            const double tau = e.red ? R - ph : (C - ph) + R;
            const double delta = tau / ht;
            const double fl = std::floor(delta);
            long c = m + (long)fl;
            double f = delta - fl;
            if (c > n_t - 2) {
                f += (double)(c - (n_t - 2));
                c = n_t - 2;
            }
            if (f <= 1.0) {
                e.wc = (int32_t)c;
                e.wf = f;
                e.tau = tau;
                e.wcost = (float)(wt * tau);
                e.wf32 = (float)f;
                e.wg32 = (float)(1.0 - f);
                e.ncyc = (int32_t)std::nearbyint((t0_abs + tm - O - ph) / C) + e.yel;
            }
        }
        out[m] = e;
    }
}

// Bound on |r_xi' - j| over every node and control of every stage.  For a
// speed node and a motor torque the battery current does not depend on the
// engine torque; the step time is longest for the lowest engine torque on the
// steepest uphill grade (least tractive force, most road load), and the
// current is largest in magnitude at the lowest open-circuit voltage.
int soc_shift_bound(const DevInst &P, const dp_problem_desc &d)
{
    double gmax = -1.0e300;
    for (int k = 0; k < d.n_stages; k++) gmax = std::max(gmax, d.grade[k]);
    const double cosa = 1.0 / std::sqrt(1.0 + gmax * gmax), sina = gmax * cosa;
    const double xis[2] = {d.soc_lo, d.soc_hi};
    double smax = 0.0;
    for (int i = 0; i < P.n_v; i++) {
        const double v = P.v_lo + i * P.hv;
        if (!(v > 0.0)) continue;
        for (int b = 0; b < P.n_m; b++) {
            const double Tm = P.m_lo + b * P.hm;
            const double Ftr = P.eta * (P.e_lo + Tm) * P.ig / P.rw;
            const double Froad = P.M * P.g * (P.Crr * cosa + sina) + 0.5 * P.rho * P.CdA * v * v;
            const double q = v * v + 2.0 * P.ds * (Ftr - Froad) / P.M;
            const double v1 = q > 0.0 ? std::sqrt(q) : 0.0;
            const double dt = 2.0 * P.ds / (v + v1);
            const double Pm = Tm * v * P.ig / P.rw;
            const double Pb = Pm >= 0.0 ? Pm / P.etam : Pm * P.etam;
            for (double xi : xis) {
                double I;
                if (!battery_current(P, Pb, xi, I)) continue;
                smax = std::max(smax, dt * std::fabs(I) / (P.Cnom * P.hs));
            }
        }
    }
    if (smax > 1.0e6) smax = 1.0e6;
    return (int)std::ceil(smax) + 1;
}

}  // namespace

extern "C" {

const char *dp_status_string(int code)
{
    switch (code) {
    case DP_OK: return "ok";
    case DP_EINVAL: return "invalid argument";
    case DP_ENOMEM: return "out of memory";
    case DP_EDEVICE: return "device error";
    case DP_EINFEASIBLE: return "infeasible";
    case DP_ESTATE: return "call out of order";
    case DP_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

int dp_last_error(char *buf, size_t n)
{
    if (!buf || n == 0) return DP_EINVAL;
    std::snprintf(buf, n, "%s", g_last_error.c_str());
    return DP_OK;
}

// Rounds of the batched solve.  Round r holds stage N_b - 1 - r of every
// instance b with N_b > r, so one launch per kernel serves all instances of
// a round.  Grouped-sweep jobs are grouped by kernel class (SoC tile, LDS
// pitch, block size) and put in decreasing order of work per item, so the
// longest items are taken first.  Control slices are chosen per round: a
// round with few (speed node, tile) pairs is split until it has about eight
// items per CU.  Appends the partial-result buffers and the queue counters to
// the scratch layout and uploads the tables.
static int plan_rounds(dp_plan *p, size_t scr)
{
    const int n_inst = (int)p->inst.size();
    int maxN = 0;
    for (const Inst &I : p->inst) maxN = std::max(maxN, I.N);
    p->rounds.assign(maxN, Round{});
    std::vector<int> ib;
    int q_slot = 0;
    std::vector<int> cur_set(n_inst, -1);   // table set holding each instance's latest tables
    // about 20 items per CU, so that the last items of a launch are short
    // against the whole; a slice costs a partial-result store and a share
    // of the combine (measured best: 8-10 slices on realistic_2km, 4 on
    // large_3km).  Items of 16-row tiles carry twice the rows and three of
    // their workgroups fit per CU instead of five: about 12 per CU keeps
    // some four items per resident workgroup (measured best 10-12 slices
    // on realistic_2km with 16-row tiles).
    for (int r = 0; r < maxN; r++) {
        Round &R = p->rounds[r];
        long base = 0;
        std::vector<int> members;
        for (int b = 0; b < n_inst; b++) {
            const Inst &I = p->inst[b];
            if (I.N <= r) continue;
            if (I.sweep == 2) {
                members.push_back(b);
                base += (long)I.P.n_v * ((I.P.n_s + I.jt - 1) / I.jt);
            } else {
                R.simple.push_back(b);
            }
        }
        bool wide = !members.empty();
        for (int b : members) wide = wide && p->inst[b].jt > 8;
        const long target = (wide ? 12L : 20L) * p->n_cu;
        const int ns_round = (int)std::min<long>(16, std::max<long>(1, (target + base - 1) / std::max(1L, base)));
        struct Tmp { int b, cls_jt, cls_pitch, cls_threads, ns; double cost; };
        std::vector<Tmp> t;
        for (int b : members) {
            Inst &I = p->inst[b];
            int ns = I.split_opt > 0 ? I.split_opt : ns_round;
            ns = std::max(1, std::min(ns, std::min(16, I.P.n_u)));
            I.nsplit = std::max(I.nsplit, ns);
            const int pitch = sweep_pitch(I.P.n_t);
            const int threads = sweep_threads(I.jt, I.P.n_t);
            t.push_back({b, I.jt, pitch, threads, ns, (double)I.P.n_u / ns});
        }
        std::stable_sort(t.begin(), t.end(), [](const Tmp &x, const Tmp &y) {
            if (x.cls_jt != y.cls_jt) return x.cls_jt > y.cls_jt;
            if (x.cls_pitch != y.cls_pitch) return x.cls_pitch > y.cls_pitch;
            if (x.cls_threads != y.cls_threads) return x.cls_threads > y.cls_threads;
            return x.cost > y.cost;
        });
        R.job_begin = (int)p->jobs.size();
        R.njobs = (int)t.size();
        for (size_t q = 0; q < t.size(); q++) {
            Inst &I = p->inst[t[q].b];
            const int k = I.N - 1 - r;
            StageJob j;
            std::memset(&j, 0, sizeof j);
            j.inst = t[q].b;
            j.k = k;
            j.jt = I.jt;
            j.ntiles = (I.P.n_s + I.jt - 1) / I.jt;
            j.nsplit = t[q].ns;
            j.H = I.H;
            j.rw = sweep_rows(I.jt, I.H);
            j.nitems = I.P.n_v * j.ntiles * j.nsplit;
            const int L = I.light_of_stage[k];
            j.tl = L >= 0 ? (int)(I.tl_dev_off + (size_t)L * I.P.n_t) : -1;
            const bool all = (p->flags & DP_STORE_ALL_V) != 0;
            j.jn = (long long)(I.J_off + sizeof(float) * I.S * (size_t)(all ? k + 1 : ((k + 1) & 1)));
            j.jk = (long long)(I.J_off + sizeof(float) * I.S * (size_t)(all ? k : (k & 1)));
            j.pik = (long long)(I.pi_off + sizeof(int16_t) * I.S * (size_t)k);
            // the previous round's set when stage k's tables equal stage k+1's,
            // else the other set (its last reader precedes this round)
            const bool reuse = cur_set[t[q].b] >= 0 && I.same_tables[k];
            const int tset = reuse ? cur_set[t[q].b] : (cur_set[t[q].b] < 0 ? 0 : 1 - cur_set[t[q].b]);
            cur_set[t[q].b] = tset;
            const long long set = (long long)(tset * I.tab_stride);
            j.st = (long long)I.scr_st + set;
            j.nf = (long long)I.scr_nf + set;
            j.rec = (long long)I.scr_rec + set;
            j.pw = (long long)I.scr_pw + set;
            if (I.job_of_k.empty()) I.job_of_k.assign(I.N, -1);
            I.job_of_k[k] = (int)p->jobs.size();
            p->jobs.push_back(j);
            if (!reuse) {
                if (R.nbjobs == 0) R.bjob_begin = (int)p->bjobs.size();
                R.nbjobs++;
                R.bmax_nv = std::max(R.bmax_nv, I.P.n_v);
                R.bmax_records = std::max(R.bmax_records, (long)I.P.n_v * I.P.n_u * j.ntiles * I.jt);
                p->bjobs.push_back(j);
            }
            R.max_nv = std::max(R.max_nv, I.P.n_v);
            R.max_records = std::max(R.max_records, (long)I.P.n_v * I.P.n_u * j.ntiles * I.jt);
            R.max_nodes = std::max(R.max_nodes, (long)I.S);
            R.any_split = R.any_split || j.nsplit > 1;
            // a new launch starts where the class changes
            if (q == 0 || t[q].cls_jt != t[q - 1].cls_jt || t[q].cls_pitch != t[q - 1].cls_pitch ||
                t[q].cls_threads != t[q - 1].cls_threads) {
                SweepLaunch L2;
                L2.jt = t[q].cls_jt;
                L2.pitch = t[q].cls_pitch;
                L2.threads = t[q].cls_threads;
                L2.job_begin = R.job_begin + (int)q;
                L2.q_slot = q_slot++;
                R.sweeps.push_back(L2);
            }
            SweepLaunch &S = R.sweeps.back();
            S.njobs++;
            S.items += j.nitems;
            S.work += (double)j.nitems * ((double)I.P.n_u / j.nsplit) * I.jt * t[q].cls_threads;
            S.lds = std::max(S.lds, lds_sweep_bytes(I.jt, I.H, I.P.n_t));
        }
        for (SweepLaunch &S : R.sweeps) {
            S.lds += lds_job_index_bytes(S.njobs);
            size_t wg = (size_t)p->lds_per_cu / S.lds;
            const int waves = S.threads / 64;
            if (wg * waves > 32) wg = 32 / waves;
            // the smallest per-CU workgroup count any job of the launch asks for
            for (int q = 0; q < S.njobs; q++) {
                const int w = p->inst[p->jobs[S.job_begin + q].inst].wg_opt;
                if (w > 0 && (size_t)w < wg) wg = w;
            }
            if (wg < 1) wg = 1;
            S.grid = (int)(wg * (size_t)p->n_cu);
            S.ib_off = ib.size();
            int run = 0;
            for (int q = 0; q < S.njobs; q++) {
                ib.push_back(run);
                run += p->jobs[S.job_begin + q].nitems;
            }
            ib.push_back(run);
        }
        // largest launch first: it starts on the main stream, the others beside it
        std::stable_sort(R.sweeps.begin(), R.sweeps.end(),
                         [](const SweepLaunch &x, const SweepLaunch &y) { return x.work > y.work; });
    }
    // partial results of control slices, sized for the largest slice count
    for (Inst &I : p->inst) {
        if (I.sweep != 2 || I.nsplit <= 1) continue;
        I.scr_pv = scr;
        scr += align_up(sizeof(float) * I.S * I.nsplit, 256);
        I.scr_pu = scr;
        scr += align_up(sizeof(int16_t) * I.S * I.nsplit, 256);
    }
    for (StageJob &j : p->jobs) {
        j.pv = (long long)p->inst[j.inst].scr_pv;
        j.pu = (long long)p->inst[j.inst].scr_pu;
    }
    for (StageJob &j : p->bjobs) {
        j.pv = (long long)p->inst[j.inst].scr_pv;
        j.pu = (long long)p->inst[j.inst].scr_pu;
    }
    p->n_q_slots = q_slot + 1;
    p->scr_q = scr;
    scr += align_up(sizeof(int) * 8 * (size_t)p->n_q_slots, 256);
    p->scr_gpart = scr;   // adjoint: per-workgroup partial gradient sums
    scr += align_up(sizeof(double) * 5 * 1024, 256);
    int max_N = 1;
    for (const Inst &I : p->inst) max_N = std::max(max_N, I.N);
    p->scr_gstage = scr;  // adjoint: per-(stage, workgroup) C_rr shares for the grade sensitivities
    scr += align_up(sizeof(double) * adjoint_grade_slots() * (size_t)max_N, 256);
    int max_L = 1;
    for (const Inst &I : p->inst) max_L = std::max(max_L, I.n_lights);
    p->scr_gspat = scr;   // adjoint: per-(signal, workgroup) pairs for the signal-timing sensitivities
    scr += align_up(sizeof(double) * 2 * adjoint_grade_slots() * (size_t)max_L, 256);
    size_t max_tab = 0;
    for (const Inst &I : p->inst) max_tab = std::max(max_tab, adjoint_table_bytes(I.P));
    p->scr_adjtab = scr;  // adjoint: the stage table of the instance being differentiated
    scr += align_up(max_tab, 256);
    p->bytes_scratch = scr;

    const size_t b_inst = align_up(sizeof(DevInst) * n_inst, 256);
    const size_t b_jobs = align_up(sizeof(StageJob) * std::max<size_t>(1, p->jobs.size()), 256);
    const size_t b_ib = align_up(sizeof(int) * std::max<size_t>(1, ib.size()), 256);
    const size_t b_bj = align_up(sizeof(StageJob) * std::max<size_t>(1, p->bjobs.size()), 256);
    // the error word, then one evaluation counter per instance (zeroed here)
    const size_t b_cnt = align_up(sizeof(unsigned long long) * (1 + (size_t)n_inst), 256);
    const size_t b_roll = align_up(sizeof(long long) * 4 * (size_t)n_inst, 256);
    const size_t b_all = b_inst + b_jobs + b_ib + b_bj + b_cnt + b_roll;
    hipError_t e = hipMalloc(&p->dev_tables, b_all);
    if (e != hipSuccess) return fail(DP_ENOMEM, "hipMalloc of %zu table bytes: %s", b_all, hipGetErrorString(e));
    std::vector<unsigned char> host(b_all, 0);
    for (int b = 0; b < n_inst; b++) std::memcpy(host.data() + sizeof(DevInst) * b, &p->inst[b].P, sizeof(DevInst));
    if (!p->jobs.empty()) std::memcpy(host.data() + b_inst, p->jobs.data(), sizeof(StageJob) * p->jobs.size());
    if (!ib.empty()) std::memcpy(host.data() + b_inst + b_jobs, ib.data(), sizeof(int) * ib.size());
    if (!p->bjobs.empty())
        std::memcpy(host.data() + b_inst + b_jobs + b_ib, p->bjobs.data(), sizeof(StageJob) * p->bjobs.size());
    char *d = (char *)p->dev_tables;
    p->dev_insts = (DevInst *)d;
    p->dev_jobs = (StageJob *)(d + b_inst);
    p->dev_ib = (int *)(d + b_inst + b_jobs);
    p->dev_bjobs = (StageJob *)(d + b_inst + b_jobs + b_ib);
    p->dev_err = (int *)(d + b_inst + b_jobs + b_ib + b_bj);
    p->dev_count = (unsigned long long *)(d + b_inst + b_jobs + b_ib + b_bj) + 1;
    p->dev_roll = (long long *)(d + b_inst + b_jobs + b_ib + b_bj + b_cnt);
    {
        long long *roll = (long long *)(host.data() + b_inst + b_jobs + b_ib + b_bj + b_cnt);
        const bool all = (p->flags & DP_STORE_ALL_V) != 0;
        for (int b = 0; b < n_inst; b++) {
            const Inst &I = p->inst[b];
            roll[b] = (long long)I.pi_off;
            roll[n_inst + b] = (long long)I.traj_off;
            roll[2 * n_inst + b] = (long long)(I.J_off + sizeof(float) * I.S);     // J_1: slab 1 in both layouts
            roll[3 * n_inst + b] = (long long)(I.J_off + sizeof(float) * I.S * (size_t)(all ? I.N : (I.N & 1)));
            p->max_slab = std::max(p->max_slab, (long)I.S);
        }
    }
    if ((e = hipMemcpy(p->dev_tables, host.data(), host.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "table upload");
    return DP_OK;
}

// Persistent batched sweep.  Each instance's stages get their tables from
// one table set per run of stages with equal tables (built together before
// the sweep); instances are grouped into kernel classes (SoC tile and waves
// per workgroup, the LDS pitch of the class's widest time grid) and, within
// a class, dealt to the XCDs by decreasing work; each XCD queue lists its
// instances' stage jobs round by round (stage N_b - 1 - r in round r),
// larger items first inside a round.  No control slices: the instances of a
// batch already give every CU work.  Falls back to rounds (returns DP_OK
// with persist unset) when an instance is on the simple sweep or the extra
// table sets would take more than half of the free device memory.
// Workgroups of a persistent class per those it needs resident (measured on
// 256 heterogeneous solves: 1.0 -> 1924 ms, 1.5 -> 1607 ms, 2.5 -> 1513 ms).
constexpr double kPersistOversub = 2.5;

static int plan_persist(dp_plan *p)
{
    const int n_inst = (int)p->inst.size();
    for (const Inst &I : p->inst)
        if (I.sweep != 2) return DP_OK;
    p->n_xcd = std::max(1, p->n_cu / 32);
    // table sets: per instance, one per run of stages with equal tables
    std::vector<std::vector<int>> set_of(n_inst);
    std::vector<std::vector<int>> set_k(n_inst);          // first (highest) stage of each set
    size_t extra = 0;
    for (int b = 0; b < n_inst; b++) {
        const Inst &I = p->inst[b];
        set_of[b].assign(I.N, 0);
        int sidx = 0;
        set_k[b].push_back(I.N - 1);
        for (int k = I.N - 2; k >= 0; k--) {
            if (!I.same_tables[k]) {
                sidx++;
                set_k[b].push_back(k);
            }
            set_of[b][k] = sidx;
        }
        if (sidx + 1 > 2) extra += (size_t)(sidx + 1 - 2) * I.tab_stride;
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return DP_OK;
    }
    if (extra > free_b / 2) return DP_OK;
    size_t scr = align_up(p->bytes_scratch, 256);
    std::vector<size_t> xset(n_inst, 0);
    for (int b = 0; b < n_inst; b++) {
        const Inst &I = p->inst[b];
        const int ns = (int)set_k[b].size();
        if (ns > 2) {
            xset[b] = scr;
            scr += (size_t)(ns - 2) * I.tab_stride;
            scr = align_up(scr, 256);
        }
    }
    auto set_base = [&](int b, int sidx) -> long long {
        const Inst &I = p->inst[b];
        return sidx < 2 ? (long long)(sidx * I.tab_stride) : (long long)(xset[b] + (sidx - 2) * I.tab_stride - I.scr_st);
    };
    auto stage_job = [&](int b, int k) {
        const Inst &I = p->inst[b];
        StageJob j;
        std::memset(&j, 0, sizeof j);
        j.inst = b;
        j.k = k;
        j.jt = I.jt;
        j.ntiles = (I.P.n_s + I.jt - 1) / I.jt;
        j.nsplit = 1;
        j.H = I.H;
        j.rw = sweep_rows(I.jt, I.H);
        j.nitems = I.P.n_v * j.ntiles;
        const int L = I.light_of_stage[k];
        j.tl = L >= 0 ? (int)(I.tl_dev_off + (size_t)L * I.P.n_t) : -1;
        const bool all = (p->flags & DP_STORE_ALL_V) != 0;
        j.jn = (long long)(I.J_off + sizeof(float) * I.S * (size_t)(all ? k + 1 : ((k + 1) & 1)));
        j.jk = (long long)(I.J_off + sizeof(float) * I.S * (size_t)(all ? k : (k & 1)));
        j.pik = (long long)(I.pi_off + sizeof(int16_t) * I.S * (size_t)k);
        const long long sb = set_base(b, set_of[b][k]);
        j.st = (long long)I.scr_st + sb;
        j.nf = (long long)I.scr_nf + sb;
        j.rec = (long long)I.scr_rec + sb;
        j.pw = (long long)I.scr_pw + sb;
        j.pv = j.pu = 0;
        return j;
    };
    // table builds: one job per set
    std::vector<StageJob> pb;
    for (int b = 0; b < n_inst; b++) {
        const Inst &I = p->inst[b];
        for (int k : set_k[b]) {
            pb.push_back(stage_job(b, k));
            p->pb_max_nv = std::max(p->pb_max_nv, I.P.n_v);
            p->pb_max_records = std::max(p->pb_max_records, (long)I.P.n_v * I.P.n_u * pb.back().ntiles * I.jt);
        }
    }
    p->n_pbjobs = (int)pb.size();
    // classes by (tile, block)
    std::vector<int> cls_of(n_inst, -1);
    for (int b = 0; b < n_inst; b++) {
        const Inst &I = p->inst[b];
        const int threads = sweep_threads(I.jt, I.P.n_t);
        int c = -1;
        for (size_t q = 0; q < p->pclasses.size(); q++)
            if (p->pclasses[q].jt == I.jt && p->pclasses[q].threads == threads) c = (int)q;
        if (c < 0) {
            dp_plan::PClass C;
            C.jt = I.jt;
            C.threads = threads;
            p->pclasses.push_back(C);
            c = (int)p->pclasses.size() - 1;
        }
        cls_of[b] = c;
        dp_plan::PClass &C = p->pclasses[c];
        C.members.push_back(b);
        C.pitch = std::max(C.pitch, sweep_pitch(I.P.n_t));
    }
    for (dp_plan::PClass &C : p->pclasses) {
        if (C.pitch > 512 || C.threads > 1024) {
            p->pclasses.clear();
            return DP_OK;
        }
        for (int b : C.members) C.lds = std::max(C.lds, lds_sweep_bytes_p(C.jt, p->inst[b].H, C.pitch, C.threads));
        if (C.lds > (size_t)p->lds_per_cu) {
            p->pclasses.clear();
            return DP_OK;
        }
    }
    // Instances to XCDs, the longest first onto the least-loaded XCD, over
    // all classes together (a class's workgroups are spread evenly over the
    // XCDs, its instances are not).  Work is counted in wave time: node-control
    // evaluations over the time nodes, times the waves of a workgroup (a wave
    // covers 63 time nodes, however few of them are on the grid).
    std::vector<double> wt(n_inst);
    for (int b = 0; b < n_inst; b++) {
        const Inst &I = p->inst[b];
        wt[b] = (double)I.evals * (double)(sweep_threads(I.jt, I.P.n_t) / 64) / (double)I.P.n_t;
    }
    std::vector<int> order(n_inst);
    for (int b = 0; b < n_inst; b++) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return wt[a] > wt[b]; });
    std::vector<int> xcd_of(n_inst, 0);
    std::vector<double> load(p->n_xcd, 0.0);
    for (int b : order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        xcd_of[b] = x;
        load[x] += wt[b];
    }
    // queues
    std::vector<PJob> pj;
    std::vector<int> pint;
    int claim = 0;
    const int cu_per_xcd = std::max(1, p->n_cu / p->n_xcd);
    for (int c = 0; c < (int)p->pclasses.size(); c++) {
        dp_plan::PClass &C = p->pclasses[c];
        std::vector<std::vector<int>> xq(p->n_xcd);
        std::vector<double> wx(p->n_xcd, 0.0);
        for (int b : order)
            if (cls_of[b] == c) {
                xq[xcd_of[b]].push_back(b);
                wx[xcd_of[b]] += wt[b];
                C.work += wt[b];
            }
        C.xjb_off = (int)pint.size();
        std::vector<int> bounds, totals;
        int max_total = 1;
        for (int x = 0; x < p->n_xcd; x++) {
            bounds.push_back((int)pj.size());
            int maxN = 0;
            for (int b : xq[x]) maxN = std::max(maxN, p->inst[b].N);
            int item0 = 0;
            for (int r = 0; r < maxN; r++) {
                std::vector<int> rb;
                for (int b : xq[x])
                    if (p->inst[b].N > r) rb.push_back(b);
                std::stable_sort(rb.begin(), rb.end(), [&](int a, int b) {
                    return (double)p->inst[a].P.n_u * p->inst[a].P.n_t > (double)p->inst[b].P.n_u * p->inst[b].P.n_t;
                });
                for (int b : rb) {
                    PJob e;
                    std::memset(&e, 0, sizeof e);
                    e.j = stage_job(b, p->inst[b].N - 1 - r);
                    e.need = r * e.j.nitems;
                    e.item0 = item0;
                    item0 += e.j.nitems;
                    pj.push_back(e);
                }
            }
            totals.push_back(item0);
            max_total = std::max(max_total, item0);
        }
        bounds.push_back((int)pj.size());
        pint.insert(pint.end(), bounds.begin(), bounds.end());
        pint.insert(pint.end(), totals.begin(), totals.end());
        C.claim_off = claim;
        claim += p->n_xcd;
        // workgroups per XCD: the class's share of the work of an XCD times
        // the workgroups of the class an XCD holds, for the XCD that needs
        // the most (the classes run side by side; elsewhere the surplus
        // workgroups find their queue drained and leave), times
        // kPersistOversub: workgroups beyond the resident ones start as
        // those of classes that finish early leave, so the last classes
        // still fill the chip
        int per_cu = persist_blocks_per_cu(C.jt, C.pitch, C.threads, C.lds);
        if (per_cu < 1) {
            per_cu = (int)std::max<size_t>(1, (size_t)p->lds_per_cu / C.lds);
            per_cu = std::max(1, std::min(per_cu, 32 / std::max(1, C.threads / 64)));
        }
        long per_x = 1;
        for (int x = 0; x < p->n_xcd; x++)
            if (wx[x] > 0.0 && load[x] > 0.0)
                per_x = std::max<long>(per_x, (long)std::ceil(kPersistOversub * wx[x] / load[x] * per_cu * cu_per_xcd));
        per_x = std::min<long>(per_x, max_total);
        C.grid = (int)(per_x * p->n_xcd);
    }
    // device tables
    const size_t b_pj = align_up(sizeof(PJob) * std::max<size_t>(1, pj.size()), 256);
    const size_t b_pi = align_up(sizeof(int) * std::max<size_t>(1, pint.size()), 256);
    const size_t b_pb = align_up(sizeof(StageJob) * std::max<size_t>(1, pb.size()), 256);
    hipError_t e = hipMalloc(&p->dev_ptables, b_pj + b_pi + b_pb);
    if (e != hipSuccess) return fail(DP_ENOMEM, "hipMalloc of %zu persistent-table bytes: %s", b_pj + b_pi + b_pb,
                                     hipGetErrorString(e));
    std::vector<unsigned char> host(b_pj + b_pi + b_pb, 0);
    if (!pj.empty()) std::memcpy(host.data(), pj.data(), sizeof(PJob) * pj.size());
    if (!pint.empty()) std::memcpy(host.data() + b_pj, pint.data(), sizeof(int) * pint.size());
    if (!pb.empty()) std::memcpy(host.data() + b_pj + b_pi, pb.data(), sizeof(StageJob) * pb.size());
    char *d = (char *)p->dev_ptables;
    p->dev_pjobs = (PJob *)d;
    p->dev_pint = (int *)(d + b_pj);
    p->dev_pbjobs = (StageJob *)(d + b_pj + b_pi);
    if ((e = hipMemcpy(p->dev_ptables, host.data(), host.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "persistent table upload");
    // counters: claims of every class, then done per instance
    p->scr_pc = scr;
    p->done_off = claim;
    p->n_pc = (long)claim + n_inst;
    scr += align_up(sizeof(int) * (size_t)p->n_pc, 256);
    p->bytes_scratch = scr;
    if (p->flags & DP_STALL_TEST) p->spin_limit = 1000;
    p->persist = true;
    return DP_OK;
}

int dp_build_problem(const dp_problem_desc *desc, int32_t n_inst, const dp_options *opt, int device, dp_plan **out)
{
    if (!out) return fail(DP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!desc || n_inst < 1) return fail(DP_EINVAL, "need at least one problem description");
    if (opt && (opt->flags & ~(DP_STORE_ALL_V | DP_TIMING | DP_GRAPH | DP_ROUNDS | DP_STALL_TEST | DP_ADJOINT_WIDE)))
        return fail(DP_EINVAL, "unknown option flags");
    if (opt && (opt->flags & DP_GRAPH) && (opt->flags & DP_TIMING))
        return fail(DP_EINVAL, "option flags DP_GRAPH and DP_TIMING exclude each other");
    if (n_inst > 1024) return fail(DP_EUNSUPPORTED, "at most 1024 instances per plan");
    auto check_opt = [](int kernel, const int32_t *t, bool t3) -> int {
        if (kernel < 0 || kernel > 2) return fail(DP_EINVAL, "unknown sweep kernel %d", kernel);
        if (t[0] != 0 && t[0] != 4 && t[0] != 8 && t[0] != 16) return fail(DP_EINVAL, "tile[0] must be 0, 4, 8 or 16");
        if (t[1] < 0 || t[1] > 16 || t[2] < 0 || t[2] > 32 || (t3 && t[3] != 0))
            return fail(DP_EINVAL, "tile[1] must be in [0, 16], tile[2] in [0, 32], tile[3] zero");
        return DP_OK;
    };
    if (opt) {
        int rc = check_opt(opt->kernel, opt->tile, true);
        if (rc) return rc;
        if (opt->inst_opt)
            for (int b = 0; b < n_inst; b++)
                if ((rc = check_opt(opt->inst_opt[4 * b], opt->inst_opt + 4 * b + 1, false)))
                    return fail(rc, "instance %d: %s", b, std::string(g_last_error).c_str());
    }
    for (int b = 0; b < n_inst; b++) {
        int rc = validate(desc[b], b);
        if (rc) return rc;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(DP_EDEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(DP_EINVAL, "device %d out of range", device);
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");

    dp_plan *p = new (std::nothrow) dp_plan;
    if (!p) return fail(DP_ENOMEM, "host allocation");
    p->device = device;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
            p->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
            p->lds_per_cu = prop.sharedMemPerBlock > 0 ? (int)prop.sharedMemPerBlock : 64 * 1024;
        }
    }
    if (opt) p->opt = *opt;
    p->flags = p->opt.flags;
    p->inst.resize(n_inst);

    // host tables and the size of one device parameter block
    size_t param_bytes = 0, n_tl = 0;
    std::vector<std::vector<double>> cosa(n_inst), sina(n_inst), vmax(n_inst), lc(n_inst), lr(n_inst), lo(n_inst),
        ly(n_inst);
    for (int b = 0; b < n_inst; b++) {
        const dp_problem_desc &d = desc[b];
        Inst &I = p->inst[b];
        const int N = d.n_stages;
        I.N = N;
        I.S = (size_t)d.n_v * d.n_soc * d.n_t;
        cosa[b].resize(N);
        sina[b].resize(N);
        for (int k = 0; k < N; k++) {
            const double G = d.grade[k];
            cosa[b][k] = 1.0 / std::sqrt(1.0 + G * G);
            sina[b][k] = G * cosa[b][k];
        }
        vmax[b].resize(N + 1);
        for (int k = 0; k <= N; k++) vmax[b][k] = d.v_max ? d.v_max[k] : d.v_hi;
        I.light_of_stage.assign(N + 1, -1);
        I.n_lights = d.n_lights;
        for (int L = 0; L < d.n_lights; L++) {
            I.light_of_stage[d.light_stage[L]] = L;
            lc[b].push_back(d.light_cycle[L]);
            lr[b].push_back(d.light_red[L]);
            lo[b].push_back(d.light_offset[L]);
            ly[b].push_back(d.light_yellow ? d.light_yellow[L] : 0.0);
        }
        param_bytes += align_up(sizeof(double) * (2 * N + (N + 1) + 4 * d.n_lights + 3), 256);
        param_bytes += align_up(sizeof(int) * (N + 1), 256);
        if (d.terminal_V) param_bytes += align_up(sizeof(float) * I.S, 256);
        I.tl_dev_off = n_tl;
        n_tl += (size_t)d.n_lights * d.n_t;
    }
    const size_t tl_bytes = align_up(sizeof(TLEntry) * (n_tl ? n_tl : 1), 256);
    if ((e = hipMalloc(&p->dev_params, param_bytes + tl_bytes)) != hipSuccess) {
        delete p;
        return fail(DP_ENOMEM, "hipMalloc of %zu parameter bytes: %s", param_bytes + tl_bytes, hipGetErrorString(e));
    }
    std::vector<unsigned char> host(param_bytes + tl_bytes, 0);
    size_t off = 0;
    char *dev = (char *)p->dev_params;
    p->dev_tl = (TLEntry *)(dev + param_bytes);
    TLEntry *host_tl = (TLEntry *)(host.data() + param_bytes);
    auto put = [&](const void *src, size_t bytes) -> char * {
        std::memcpy(host.data() + off, src, bytes);
        char *d = dev + off;
        off += align_up(bytes, 256);
        return d;
    };
    // device-resident terminal tables, copied after the host block
    struct DevCopy {
        char *dst;
        const void *src;
        size_t bytes;
    };
    std::vector<DevCopy> dev_copies;
    auto put_device = [&](const void *src, size_t bytes) -> char * {
        char *d = dev + off;
        dev_copies.push_back({d, src, bytes});
        off += align_up(bytes, 256);
        return d;
    };
    size_t J_off = 0, pi_off = 0, traj_off = 0, scr = 0;
    for (int b = 0; b < n_inst; b++) {
        const dp_problem_desc &d = desc[b];
        Inst &I = p->inst[b];
        const int N = d.n_stages;
        DevInst &P = I.P;
        std::memset(&P, 0, sizeof P);
        P.N = N;
        P.n_v = d.n_v;
        P.n_s = d.n_soc;
        P.n_t = d.n_t;
        P.n_e = d.n_te;
        P.n_m = d.n_tm;
        P.n_u = d.n_te * d.n_tm;
        P.wait = (d.flags & DP_WAIT_AT_RED) ? 1 : 0;
        P.zero_row = d.v_lo == 0.0 ? 0 : -1;
        P.ds = d.ds;
        P.v_lo = d.v_lo;
        P.s_lo = d.soc_lo;
        P.v_hi = d.v_hi;
        P.s_hi = d.soc_hi;
        P.t_f = d.t_f;
        P.hv = gstep(d.v_lo, d.v_hi, d.n_v);
        P.hs = gstep(d.soc_lo, d.soc_hi, d.n_soc);
        P.ht = gstep(0.0, d.t_f, d.n_t);
        P.he = gstep(d.te_lo, d.te_hi, d.n_te);
        P.hm = gstep(d.tm_lo, d.tm_hi, d.n_tm);
        P.e_lo = d.te_lo;
        P.m_lo = d.tm_lo;
        P.M = d.theta[0];
        P.CdA = d.theta[1];
        P.Crr = d.theta[2];
        P.wt = d.theta[3];
        P.wsoc = d.theta[4];
        const double *K = d.konst;
        P.g = K[0];
        P.rho = K[1];
        P.rw = K[2];
        P.ig = K[3];
        P.eta = K[4];
        P.etam = K[5];
        P.Cnom = K[6];
        P.Voc0 = K[7];
        P.Voc1 = K[8];
        P.Rb = K[9];
        P.amin = K[10];
        P.amax = K[11];
        P.xiref = K[12];
        P.Jinf = K[13];
        P.peng = K[14];
        P.pbsg = K[15];
        for (int q = 0; q < 6; q++) P.q[q] = d.fuel[q];
        P.v0 = d.v0;
        P.soc0 = d.soc0;
        P.t0_abs = d.t0_abs;
        std::vector<double> dbl;
        dbl.insert(dbl.end(), cosa[b].begin(), cosa[b].end());
        dbl.insert(dbl.end(), sina[b].begin(), sina[b].end());
        dbl.insert(dbl.end(), vmax[b].begin(), vmax[b].end());
        dbl.insert(dbl.end(), lc[b].begin(), lc[b].end());
        dbl.insert(dbl.end(), lr[b].begin(), lr[b].end());
        dbl.insert(dbl.end(), lo[b].begin(), lo[b].end());
        dbl.insert(dbl.end(), ly[b].begin(), ly[b].end());
        dbl.resize(dbl.size() + 3, 0.0);
        const double *dd = (const double *)put(dbl.data(), sizeof(double) * dbl.size());
        P.cosa = dd;
        P.sina = dd + N;
        P.vmax = dd + 2 * N;
        const int nl = d.n_lights;
        P.l_cycle = dd + 3 * N + 1;
        P.l_red = P.l_cycle + nl;
        P.l_off = P.l_red + nl;
        P.l_yel = P.l_off + nl;
        P.light_of_stage = (const int *)put(I.light_of_stage.data(), sizeof(int) * (N + 1));
        P.terminal_V = !d.terminal_V ? nullptr
                       : (const float *)((d.flags & DP_TERMINAL_DEVICE) ? put_device(d.terminal_V, sizeof(float) * I.S)
                                                                       : put(d.terminal_V, sizeof(float) * I.S));
        // the stage tables of k depend on k only through the grade of step k
        // and the speed limits at k and k+1
        I.same_tables.assign(N, 0);
        for (int k = 0; k + 1 < N && !t_window.on; k++)
            I.same_tables[k] = cosa[b][k] == cosa[b][k + 1] && sina[b][k] == sina[b][k + 1] &&
                               vmax[b][k] == vmax[b][k + 1] && vmax[b][k + 1] == vmax[b][k + 2];
        I.l_cycle = lc[b];
        I.l_red = lr[b];
        I.l_off = lo[b];
        I.l_yel = ly[b];
        for (int L = 0; L < nl; L++)
            build_tl(lc[b][L], lr[b][L], lo[b][L], ly[b][L], d.t0_abs, d.t_f, d.n_t, d.theta[3],
                     host_tl + I.tl_dev_off + (size_t)L * d.n_t);

        const int nst = (p->flags & DP_STORE_ALL_V) ? N + 1 : 2;
        I.J_off = J_off;
        J_off += align_up(sizeof(float) * I.S * nst, 256);
        I.pi_off = pi_off;
        pi_off += align_up(sizeof(int16_t) * I.S * N, 256);
        I.traj_off = traj_off;
        traj_off += (size_t)(N + 1) * 8;
        // state-sweep variant: the grouped LDS kernel when its tables and
        // staged planes fit, else the simple per-node kernel
        I.H = std::max(soc_shift_bound(P, d), t_window.h_min);
        // SoC rows per workgroup: 8-row tiles when they leave five resident
        // waves per SIMD (the sweep waits on LDS and barriers, so resident
        // waves matter more than the per-tile saving), in a batch too (256
        // heterogeneous solves: 8-row tiles 1266 ms persistent, 1370 ms in
        // rounds, against 1527 / 1465 ms with 4-row tiles); else 16 rows on
        // two wave groups (single instances only), then 4, by the same bound;
        // else the tile with the most resident waves; a caller tile (or the
        // autotuner) overrides
        const double min_waves = 5.0;
        const size_t lds_cu = (size_t)p->lds_per_cu;
        // resident waves per SIMD of the grouped sweep with tile t: bounded by
        // the LDS of a CU, by 8 waves per SIMD and by the kernel's registers
        // (512 per SIMD lane, allocated in granules of 8); 0 when its
        // workgroup would exceed 1024 threads
        auto waves_per_simd = [&](int t) {
            const size_t bytes = lds_sweep_bytes(t, I.H, d.n_t);
            const int waves = sweep_threads(t, d.n_t) / 64;
            if (bytes > lds_cu || waves > 16) return 0.0;
            size_t wg = lds_cu / bytes;
            if (wg * waves > 32) wg = 32 / waves;
            const int vg = (sweep_vgprs(t, sweep_pitch(d.n_t)) + 7) / 8 * 8;
            const double w = (double)(wg * waves) / 4.0;
            return std::min(w, (double)(512 / vg));
        };
        int jt = 0;
        const int32_t *io = p->opt.inst_opt ? p->opt.inst_opt + 4 * b : nullptr;
        const int o_kernel = io && io[0] ? io[0] : p->opt.kernel;
        const int o_tile = io && io[1] ? io[1] : p->opt.tile[0];
        I.split_opt = io && io[2] ? io[2] : p->opt.tile[1];
        I.wg_opt = io && io[3] ? io[3] : p->opt.tile[2];
        if (o_tile == 4 || o_tile == 8 || o_tile == 16) {
            jt = o_tile;
            if (sweep_threads(jt, d.n_t) > 1024) jt = 8;   // 16-row tiles need n_t <= 504
        } else {
            const int cand[3] = {8, 16, 4};
            double best_w = 0.0;
            for (int t : cand) {
                if (t > 4 && d.n_soc < t) continue;
                if (t == 16 && n_inst > 1) continue;   // measured slower in a batch
                const double w = waves_per_simd(t);
                if (n_inst > 1 && t == 8 && w > 0.0) {
                    // a batch takes 8-row tiles wherever they fit: instances
                    // with one tile share the kernel classes of the persistent
                    // sweep (more classes than streams run one after another;
                    // 256 solves: 1266 ms all on 8-row tiles, 1677 ms mixed)
                    jt = t;
                    break;
                }
                if (w >= min_waves) {
                    jt = t;
                    break;
                }
                if (w > best_w) {
                    best_w = w;
                    jt = t;
                }
            }
            if (jt == 0) jt = 4;
        }
        const bool lds_fits = lds_sweep_bytes(jt, I.H, d.n_t) + lds_job_index_bytes(n_inst) <= lds_cu &&
                              sweep_threads(jt, d.n_t) <= 1024 && P.n_u <= 1024 && d.n_v - 1 <= kSortBins &&
                              I.H <= 120;   // cell offsets in the records are bytes
        I.jt = jt;
        I.sweep = o_kernel == 1 ? 1 : (lds_fits ? 2 : 1);
        if (o_kernel == 2 && !lds_fits) {
            (void)hipFree(p->dev_params);
            delete p;
            return fail(DP_EUNSUPPORTED, "instance %d: grouped sweep does not fit (n_t %d, n_u %d, H %d)", b, d.n_t,
                        P.n_u, I.H);
        }
        if (lds_fits) {
            size_t wg = lds_cu / lds_sweep_bytes(jt, I.H, d.n_t);
            const int waves = sweep_threads(jt, d.n_t) / 64;
            if (wg * waves > 32) wg = 32 / waves;
            if (I.wg_opt > 0 && (size_t)I.wg_opt < wg) wg = I.wg_opt;
            if (wg < 1) wg = 1;
            I.grid = (int)(wg * (size_t)p->n_cu);
        }
        // stage tables; the grouped sweep keeps two sets, so that the tables
        // of the next round are built while this round's sweep runs
        const size_t tab0 = scr;
        I.scr_st = scr;
        scr += align_up(sizeof(SortedEntry) * d.n_v * P.n_u, 256);
        I.scr_nf = scr;   // feasible-control counts, then the speed nodes in decreasing order of work
        scr += align_up(sizeof(int) * 2 * (size_t)d.n_v, 256);
        if (I.sweep == 2) {
            const size_t ntiles = (d.n_soc + I.jt - 1) / I.jt;
            I.scr_pw = scr;
            scr += align_up(sizeof(double) * 2 * (size_t)d.n_v * P.n_u, 256);
            I.scr_rec = scr;
            scr += align_up(sizeof(float) * (size_t)d.n_v * ntiles * P.n_u * (9 + I.jt / 4 + 2 * I.jt), 256);
            I.tab_stride = scr - tab0;
            scr += I.tab_stride;
        } else {
            I.scr_bat = scr;
            scr += align_up(sizeof(BatEntry) * ((size_t)d.n_v * P.n_u * d.n_soc + 16), 256);
        }
        I.scr_rho = scr;
        scr += align_up(sizeof(double) * I.S * 2, 256);
        I.evals = (int64_t)N * (int64_t)I.S * P.n_u;
    }
    p->bytes_J = J_off;
    p->bytes_pi = pi_off;
    if ((e = hipMemcpy(p->dev_params, host.data(), host.size(), hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(p->dev_params);
        delete p;
        return hip_fail(e, "parameter upload");
    }
    for (const DevCopy &c : dev_copies) {
        if ((e = hipMemcpy(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice)) != hipSuccess) {
            (void)hipFree(p->dev_params);
            delete p;
            return hip_fail(e, "terminal table copy");
        }
    }
    int rc = plan_rounds(p, scr);
    if (rc) {
        dp_destroy(p);
        return rc;
    }
    if (n_inst > 1 && !(p->flags & DP_ROUNDS)) {
        rc = plan_persist(p);
        if (rc) {
            dp_destroy(p);
            return rc;
        }
    }
    if (p->flags & DP_GRAPH) {
        if ((e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
            dp_destroy(p);
            return hip_fail(e, "capture stream");
        }
    }
    if (p->rounds.size() > 1) {
        e = hipStreamCreateWithFlags(&p->tstream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->tfork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->tjoin, hipEventDisableTiming);
        if (e != hipSuccess) {
            dp_destroy(p);
            return hip_fail(e, "table stream");
        }
    }
    bool multi = p->persist && p->pclasses.size() > 1;
    for (const Round &R : p->rounds) multi = multi || R.sweeps.size() > 1;
    if (multi) {
        e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
        for (int q = 0; q < dp_plan::kSide && e == hipSuccess; q++) {
            e = hipStreamCreateWithFlags(&p->side[q], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join[q], hipEventDisableTiming);
        }
        if (e != hipSuccess) {
            dp_destroy(p);
            return hip_fail(e, "side streams");
        }
    }
    *out = p;
    return DP_OK;
}

int dp_workspace_size(const dp_plan *p, size_t *bytes_J, size_t *bytes_pi, size_t *bytes_scratch)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (bytes_J) *bytes_J = p->bytes_J;
    if (bytes_pi) *bytes_pi = p->bytes_pi;
    if (bytes_scratch) *bytes_scratch = p->bytes_scratch;
    return DP_OK;
}

int dp_instance_info_get(const dp_plan *p, int32_t inst, dp_instance_info *info)
{
    if (!p || !info) return fail(DP_EINVAL, "NULL argument");
    if (inst < 0 || inst >= (int)p->inst.size()) return fail(DP_EINVAL, "instance %d out of range", inst);
    const Inst &I = p->inst[inst];
    info->n_stages = I.N;
    info->n_v = I.P.n_v;
    info->n_soc = I.P.n_s;
    info->n_t = I.P.n_t;
    info->n_u = I.P.n_u;
    info->J_offset = I.J_off;
    info->pi_offset = I.pi_off;
    info->traj_offset = I.traj_off;
    info->slab_elems = I.S;
    info->evaluations = I.evals;
    info->sweep_kernel = I.sweep;
    info->sweep_tile = I.jt;
    info->sweep_split = I.nsplit;
    info->sweep_grid = I.grid;
    info->soc_shift = I.H;
    info->sweep_persistent = 0;
    if (p->persist)
        for (const dp_plan::PClass &C : p->pclasses)
            for (int b : C.members)
                if (b == inst) {
                    info->sweep_persistent = 1;
                    info->sweep_split = 1;
                    info->sweep_grid = C.grid;
                }
    return DP_OK;
}

static float *slab_ptr(dp_plan *p, const Inst &I, void *J, int k)
{
    const int idx = (p->flags & DP_STORE_ALL_V) ? k : (k & 1);
    return (float *)((char *)J + I.J_off) + (size_t)idx * I.S;
}

static int time_begin(dp_plan *p, hipStream_t s)
{
    if (!(p->flags & DP_TIMING)) return DP_OK;
    if (p->n_ev_used + 2 > (int)p->ev.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
            return fail(DP_EDEVICE, "event creation failed");
        p->ev.push_back(a);
        p->ev.push_back(b);
    }
    (void)hipEventRecord(p->ev[p->n_ev_used], s);
    return DP_OK;
}

static void time_end(dp_plan *p, hipStream_t s)
{
    if (!(p->flags & DP_TIMING)) return;
    (void)hipEventRecord(p->ev[p->n_ev_used + 1], s);
    p->n_ev_used += 2;
}

static StageBase stage_base(dp_plan *p, void *J, void *pi, void *scratch)
{
    StageBase B;
    B.insts = p->dev_insts;
    B.jobs = p->dev_jobs;
    B.J = (char *)J;
    B.pi = (char *)pi;
    B.scr = (char *)scratch;
    B.tl = p->dev_tl;
    B.Jn = nullptr;
    B.Jk = nullptr;
    B.pik = nullptr;
    B.count = p->dev_count;
    B.err = p->dev_err;
    return B;
}

// Stage k of an instance on the simple per-node sweep.
static int enqueue_simple(dp_plan *p, const Inst &I, int k, const float *Jn, float *Jk, int16_t *pik, void *scratch,
                          hipStream_t s, bool timing = true)
{
    StageEntry *st = (StageEntry *)((char *)scratch + I.scr_st);
    BatEntry *bat = (BatEntry *)((char *)scratch + I.scr_bat);
    const int L = I.light_of_stage[k];
    const TLEntry *tl = L >= 0 ? p->dev_tl + I.tl_dev_off + (size_t)L * I.P.n_t : nullptr;
    if (launch_stage_table(I.P, k, st, bat, p->dev_count + (&I - p->inst.data()), s))
        return hip_fail(hipGetLastError(), "stage table launch");
    if (timing) {
        int rc = time_begin(p, s);
        if (rc) return rc;
    }
    if (launch_sweep(I.P, k, Jn, Jk, pik, st, bat, tl, s)) return hip_fail(hipGetLastError(), "sweep launch");
    if (timing) time_end(p, s);
    return DP_OK;
}

static int *queue_slot(dp_plan *p, void *scratch, int slot)
{
    return (int *)((char *)scratch + p->scr_q) + 8 * (size_t)slot;
}

// The terminal slabs, every round of stages, then the exact root step.
// timing = false leaves the DP_TIMING events out (they are created on demand).
static int enqueue_persist(dp_plan *p, void *J, void *pi, void *scratch, float *V0_dev, int16_t *u0_dev,
                           hipStream_t s, bool timing);

static int enqueue_solve(dp_plan *p, void *J, void *pi, void *scratch, float *V0_dev, int16_t *u0_dev, hipStream_t s,
                         bool timing = true)
{
    if (p->persist) return enqueue_persist(p, J, pi, scratch, V0_dev, u0_dev, s, timing);
    const int n_inst = (int)p->inst.size();
    if (launch_terminal_jobs(p->dev_insts, n_inst, p->max_slab, J, p->dev_roll + 3 * n_inst, p->dev_err, s))
        return hip_fail(hipGetLastError(), "terminal launch");
    if (launch_fill_i32(queue_slot(p, scratch, 0), 8L * p->n_q_slots, 0, s) ||
        launch_fill_i32((int *)p->dev_count, 2L * (long)p->inst.size(), 0, s))
        return hip_fail(hipGetLastError(), "counter reset launch");
    const StageBase base = stage_base(p, J, pi, scratch);
    bool pre = false;   // this round's grouped-sweep tables were launched on the table stream
    for (size_t r = 0; r < p->rounds.size(); r++) {
        const Round &R = p->rounds[r];
        for (int b : R.simple) {
            const Inst &I = p->inst[b];
            const int k = I.N - 1 - (int)r;
            int16_t *pik = (int16_t *)((char *)pi + I.pi_off) + (size_t)k * I.S;
            int rc = enqueue_simple(p, I, k, slab_ptr(p, I, J, k + 1), slab_ptr(p, I, J, k), pik, scratch, s, timing);
            if (rc) return rc;
        }
        if (R.njobs == 0) continue;
        StageBase B = base;
        B.jobs = p->dev_jobs + R.job_begin;
        if (pre) {
            hipError_t e = hipStreamWaitEvent(s, p->tjoin, 0);
            if (e != hipSuccess) return hip_fail(e, "table join");
        } else if (R.nbjobs > 0) {
            StageBase Bt = base;
            Bt.jobs = p->dev_bjobs + R.bjob_begin;
            if (launch_stage_jobs(Bt, R.nbjobs, R.bmax_nv, R.bmax_records, s))
                return hip_fail(hipGetLastError(), "stage table launch");
        }
        // the next round's tables (the other table set, last read by the
        // previous round, which is already ordered before this point) are
        // built beside this round's sweep
        pre = false;
        if (p->tstream && r + 1 < p->rounds.size() && p->rounds[r + 1].nbjobs > 0) {
            const Round &R1 = p->rounds[r + 1];
            StageBase B1 = base;
            B1.jobs = p->dev_bjobs + R1.bjob_begin;
            hipError_t e = hipEventRecord(p->tfork, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(p->tstream, p->tfork, 0);
            if (e != hipSuccess) return hip_fail(e, "table fork");
            if (launch_stage_jobs(B1, R1.nbjobs, R1.bmax_nv, R1.bmax_records, p->tstream))
                return hip_fail(hipGetLastError(), "stage table launch");
            if ((e = hipEventRecord(p->tjoin, p->tstream)) != hipSuccess) return hip_fail(e, "table join");
            pre = true;
        }
        // launches of different kernel classes are independent: without
        // DP_TIMING they run side by side on the plan's streams, so one
        // launch's tail overlaps the next one's start
        const bool timed = timing && (p->flags & DP_TIMING);
        const int nside = timed ? 0 : std::min<int>(dp_plan::kSide, (int)R.sweeps.size() - 1);
        if (nside > 0) {
            hipError_t e = hipEventRecord(p->fork, s);
            for (int q = 0; q < nside && e == hipSuccess; q++) e = hipStreamWaitEvent(p->side[q], p->fork, 0);
            if (e != hipSuccess) return hip_fail(e, "stream fork");
        }
        for (size_t q = 0; q < R.sweeps.size(); q++) {
            const SweepLaunch &S = R.sweeps[q];
            hipStream_t ls = (nside > 0 && q % (nside + 1) != 0) ? p->side[q % (nside + 1) - 1] : s;
            StageBase Bs = base;
            Bs.jobs = p->dev_jobs + S.job_begin;
            if (timed) {
                int rc = time_begin(p, ls);
                if (rc) return rc;
            }
            if (launch_sweep_jobs(S.jt, S.pitch, S.threads, Bs, S.njobs, p->dev_ib + S.ib_off, S.items,
                                  queue_slot(p, scratch, S.q_slot), S.grid, S.lds, ls))
                return hip_fail(hipGetLastError(), "sweep launch");
            if (timed) time_end(p, ls);
        }
        if (nside > 0) {
            hipError_t e = hipSuccess;
            for (int q = 0; q < nside && e == hipSuccess; q++) {
                e = hipEventRecord(p->join[q], p->side[q]);
                if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join[q], 0);
            }
            if (e != hipSuccess) return hip_fail(e, "stream join");
        }
        if (R.any_split && launch_combine_jobs(B, R.njobs, R.max_nodes, s))
            return hip_fail(hipGetLastError(), "combine launch");
    }
    if (launch_root_jobs(p->dev_insts, n_inst, J, p->dev_roll + 2 * n_inst, V0_dev, u0_dev, s))
        return hip_fail(hipGetLastError(), "root launch");
    return DP_OK;
}

// The persistent solve: counters cleared, terminal slabs, every table set,
// one persistent sweep per class (side by side), roots.
static int enqueue_persist(dp_plan *p, void *J, void *pi, void *scratch, float *V0_dev, int16_t *u0_dev,
                           hipStream_t s, bool timing)
{
    const int n_inst = (int)p->inst.size();
    int *pc = (int *)((char *)scratch + p->scr_pc);
    if (launch_fill_i32(pc, p->n_pc, 0, s) || launch_fill_i32((int *)p->dev_count, 2L * n_inst, 0, s))
        return hip_fail(hipGetLastError(), "counter reset launch");
    if (launch_terminal_jobs(p->dev_insts, n_inst, p->max_slab, J, p->dev_roll + 3 * n_inst, p->dev_err, s))
        return hip_fail(hipGetLastError(), "terminal launch");
    const StageBase base = stage_base(p, J, pi, scratch);
    {
        StageBase Bt = base;
        Bt.jobs = p->dev_pbjobs;
        if (launch_stage_jobs(Bt, p->n_pbjobs, p->pb_max_nv, p->pb_max_records, s))
            return hip_fail(hipGetLastError(), "stage table launch");
    }
    // with DP_TIMING the classes still run side by side: one interval from
    // before the fork to after the join
    const bool timed = timing && (p->flags & DP_TIMING);
    const int ncls = (int)p->pclasses.size();
    const int nside = std::min<int>(dp_plan::kSide, ncls - 1);
    if (timed) {
        int rc = time_begin(p, s);
        if (rc) return rc;
    }
    if (nside > 0) {
        hipError_t e = hipEventRecord(p->fork, s);
        for (int q = 0; q < nside && e == hipSuccess; q++) e = hipStreamWaitEvent(p->side[q], p->fork, 0);
        if (e != hipSuccess) return hip_fail(e, "stream fork");
    }
    for (int c = 0; c < ncls; c++) {
        const dp_plan::PClass &C = p->pclasses[c];
        hipStream_t ls = (nside > 0 && c % (nside + 1) != 0) ? p->side[c % (nside + 1) - 1] : s;
        PersistQueues Q;
        Q.jobs = p->dev_pjobs;
        Q.xjb = p->dev_pint + C.xjb_off;
        Q.xtot = p->dev_pint + C.xjb_off + p->n_xcd + 1;
        Q.claim = pc + C.claim_off;
        Q.done = pc + p->done_off;
        Q.err = p->dev_err;
        Q.n_xcd = p->n_xcd;
        Q.stall = (p->flags & DP_STALL_TEST) ? 1 : 0;
        Q.spin_limit = p->spin_limit;
        if (launch_sweep_persist(C.jt, C.pitch, C.threads, base, p->dev_insts, Q, C.grid, C.lds, ls))
            return hip_fail(hipGetLastError(), "persistent sweep launch");
    }
    if (nside > 0) {
        hipError_t e = hipSuccess;
        for (int q = 0; q < nside && e == hipSuccess; q++) {
            e = hipEventRecord(p->join[q], p->side[q]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, p->join[q], 0);
        }
        if (e != hipSuccess) return hip_fail(e, "stream join");
    }
    if (timed) time_end(p, s);
    if (launch_root_jobs(p->dev_insts, n_inst, J, p->dev_roll + 2 * n_inst, V0_dev, u0_dev, s))
        return hip_fail(hipGetLastError(), "root launch");
    return DP_OK;
}

static void drop_graph(dp_plan *p)
{
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    for (int q = 0; q < 5; q++) p->graph_key[q] = nullptr;
}

int dp_solve(dp_plan *p, void *J, void *pi, void *scratch, float *V0_dev, int16_t *u0_dev, void *stream)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (!J || !pi || !scratch || !V0_dev || !u0_dev) return fail(DP_EINVAL, "NULL buffer");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (!(p->flags & DP_GRAPH)) {
        int rc = enqueue_solve(p, J, pi, scratch, V0_dev, u0_dev, s);
        if (rc) return rc;
        p->solved = true;
        return DP_OK;
    }
    const void *key[5] = {J, pi, scratch, V0_dev, u0_dev};
    bool same = p->graph_exec != nullptr;
    for (int q = 0; q < 5; q++) same = same && key[q] == p->graph_key[q];
    if (!same) {
        drop_graph(p);
        if ((e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        const int rc = enqueue_solve(p, J, pi, scratch, V0_dev, u0_dev, p->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(p->cap_stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        p->graph = g;
        if ((e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0)) != hipSuccess) {
            p->graph_exec = nullptr;
            drop_graph(p);
            return hip_fail(e, "hipGraphInstantiate");
        }
        for (int q = 0; q < 5; q++) p->graph_key[q] = key[q];
    }
    if ((e = hipGraphLaunch(p->graph_exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    p->solved = true;
    return DP_OK;
}

// ------------------------------------------------- solve without allocation --

// Scratch of dp_solve_static, for callers that cannot allocate device memory:
// a file-scope device array, one copy on every device the library runs on,
// held until the process ends.  Host code never passes this name to a
// kernel: its device address comes from hipGetSymbolAddress, looked up once
// per device with that device current.
constexpr size_t kStaticScratchBytes = DP_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char static_scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;
static void *g_static_ptr[kMaxDevices] = {};

// Device address of static_scratch on `device` (current).
static int static_scratch_ptr(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(DP_EUNSUPPORTED, "device %d beyond the static scratch table", device);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(static_scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch address");
        g_static_ptr[device] = ptr;
    }
    *out = g_static_ptr[device];
    return DP_OK;
}

int dp_solve_static(dp_plan *p, void *J, void *pi, float *V0_dev, int16_t *u0_dev, void *stream)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (!J || !pi || !V0_dev || !u0_dev) return fail(DP_EINVAL, "NULL buffer");
    if (p->bytes_scratch > kStaticScratchBytes)
        return fail(DP_EUNSUPPORTED, "plan needs %zu scratch bytes, the static scratch holds %zu", p->bytes_scratch,
                    kStaticScratchBytes);
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    void *scratch = nullptr;
    int rc = static_scratch_ptr(p->device, &scratch);
    if (rc) return rc;
    // the same launches as dp_solve, eagerly (no graph, no timing events);
    // the queue and evaluation counters are cleared by its first fill kernel
    rc = enqueue_solve(p, J, pi, scratch, V0_dev, u0_dev, (hipStream_t)stream, false);
    if (rc) return rc;
    p->solved = true;
    return DP_OK;
}

int dp_stage(dp_plan *p, int32_t inst, int32_t k, const float *J_next, float *J_out, int16_t *pi_out, void *scratch,
             void *stream)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (inst < 0 || inst >= (int)p->inst.size()) return fail(DP_EINVAL, "instance %d out of range", inst);
    const Inst &I = p->inst[inst];
    if (k < 0 || k >= I.N) return fail(DP_EINVAL, "stage %d not in [0, N-1]", k);
    if (!J_next || !J_out || !pi_out || !scratch) return fail(DP_EINVAL, "NULL buffer");
    if (J_next == J_out) return fail(DP_EINVAL, "J_next and J_out must not alias");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (I.sweep != 2) return enqueue_simple(p, I, k, J_next, J_out, pi_out, scratch, s);
    const int idx = I.job_of_k[k];
    const StageJob &j = p->jobs[idx];
    StageBase B = stage_base(p, nullptr, nullptr, scratch);
    B.jobs = p->dev_jobs + idx;
    B.Jn = J_next;
    B.Jk = J_out;
    B.pik = pi_out;
    int *q = queue_slot(p, scratch, p->n_q_slots - 1);
    if (launch_fill_i32(q, 8, 0, s)) return hip_fail(hipGetLastError(), "queue reset launch");
    if (launch_stage_jobs(B, 1, I.P.n_v, (long)I.P.n_v * I.P.n_u * j.ntiles * I.jt, s))
        return hip_fail(hipGetLastError(), "stage table launch");
    int rc = time_begin(p, s);
    if (rc) return rc;
    const int pitch = sweep_pitch(I.P.n_t), threads = sweep_threads(I.jt, I.P.n_t);
    if (launch_sweep_jobs(I.jt, pitch, threads, B, 1, nullptr, j.nitems, q, I.grid,
                          lds_sweep_bytes(I.jt, I.H, I.P.n_t), s))
        return hip_fail(hipGetLastError(), "sweep launch");
    time_end(p, s);
    if (j.nsplit > 1 && launch_combine_jobs(B, 1, (long)I.S, s)) return hip_fail(hipGetLastError(), "combine launch");
    return DP_OK;
}

// The plan's pinned staging buffer with at least `need` bytes, free to write:
// the previous upload from it has run.
static int state_staging(dp_plan *p, size_t need)
{
    hipError_t e;
    if (p->state_pending) {
        // the staging buffer is read by the previous upload until it has run
        if ((e = hipEventSynchronize(p->state_ev)) != hipSuccess) return hip_fail(e, "state upload wait");
        p->state_pending = false;
    }
    if (need > p->state_bytes) {
        if (p->state_host) (void)hipHostFree(p->state_host);
        p->state_host = nullptr;
        p->state_bytes = 0;
        if ((e = hipHostMalloc(&p->state_host, need, hipHostMallocDefault)) != hipSuccess)
            return fail(DP_ENOMEM, "pinned staging of %zu bytes: %s", need, hipGetErrorString(e));
        p->state_bytes = need;
    }
    if (!p->state_ev && (e = hipEventCreateWithFlags(&p->state_ev, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "state event");
    return DP_OK;
}

int dp_set_state(dp_plan *p, int32_t inst, double v0, double soc0, double t0_abs, void *stream)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (inst < 0 || inst >= (int)p->inst.size()) return fail(DP_EINVAL, "instance %d out of range", inst);
    Inst &I = p->inst[inst];
    if (!(std::isfinite(v0) && v0 >= 0.0 && std::isfinite(soc0) && soc0 >= I.P.s_lo && soc0 <= I.P.s_hi &&
          std::isfinite(t0_abs)))
        return fail(DP_EINVAL, "instance %d: x0 outside the grid or not finite", inst);
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const int nl = (int)I.l_cycle.size();
    const size_t tl_n = (size_t)nl * I.P.n_t;
    const size_t need = align_up(sizeof(DevInst), 256) + sizeof(TLEntry) * (tl_n ? tl_n : 1);
    int rc = state_staging(p, need);
    if (rc) return rc;
    I.P.v0 = v0;
    I.P.soc0 = soc0;
    I.P.t0_abs = t0_abs;
    char *h = (char *)p->state_host;
    std::memcpy(h, &I.P, sizeof(DevInst));
    TLEntry *htl = (TLEntry *)(h + align_up(sizeof(DevInst), 256));
    for (int L = 0; L < nl; L++)
        build_tl(I.l_cycle[L], I.l_red[L], I.l_off[L], I.l_yel[L], t0_abs, I.P.t_f, I.P.n_t, I.P.wt,
                 htl + (size_t)L * I.P.n_t);
    e = hipMemcpyAsync(p->dev_insts + inst, h, sizeof(DevInst), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && tl_n)
        e = hipMemcpyAsync(p->dev_tl + I.tl_dev_off, htl, sizeof(TLEntry) * tl_n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(p->state_ev, s);
    if (e != hipSuccess) return hip_fail(e, "state upload");
    p->state_pending = true;
    p->solved = false;
    return DP_OK;
}


int dp_terminal_from_values(const float *src, int32_t n_v, int32_t n_soc, int32_t n_t_src, double t_f_src,
                            double t_shift, int32_t n_t_dst, double t_f_dst, double J_inf, float *dst, void *stream)
{
    if (!src || !dst) return fail(DP_EINVAL, "terminal table: NULL pointer");
    if (n_v < 1 || n_soc < 1 || n_t_src < 2 || n_t_dst < 2)
        return fail(DP_EINVAL, "terminal table: grid sizes n_v=%d n_soc=%d n_t=%d/%d", n_v, n_soc, n_t_src, n_t_dst);
    if (!(std::isfinite(t_f_src) && t_f_src > 0.0 && std::isfinite(t_f_dst) && t_f_dst > 0.0 &&
          std::isfinite(t_shift) && t_shift >= 0.0 && std::isfinite(J_inf) && J_inf > 0.0))
        return fail(DP_EINVAL, "terminal table: time grids, shift or J_inf out of range");
    const long nvs = (long)n_v * n_soc;
    const char *s0 = (const char *)src, *s1 = s0 + sizeof(float) * nvs * n_t_src;
    const char *d0 = (const char *)dst, *d1 = d0 + sizeof(float) * nvs * n_t_dst;
    if (s0 < d1 && d0 < s1) return fail(DP_EINVAL, "terminal table: src and dst overlap");
    if (launch_terminal_shift(src, nvs, n_t_src, t_f_src / (n_t_src - 1), t_shift, n_t_dst, t_f_dst / (n_t_dst - 1),
                              J_inf, dst, (hipStream_t)stream))
        return hip_fail(hipGetLastError(), "terminal table launch");
    return DP_OK;
}

int dp_rollout(dp_plan *p, const void *pi, const int16_t *u0_dev, double *traj_dev, int32_t *status_dev, void *stream)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (!pi || !u0_dev || !traj_dev || !status_dev) return fail(DP_EINVAL, "NULL buffer");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)p->inst.size();
    if (launch_rollout_jobs(p->dev_insts, n, pi, p->dev_roll, p->dev_roll + n, u0_dev, traj_dev, status_dev, s))
        return hip_fail(hipGetLastError(), "rollout launch");
    return DP_OK;
}

static int adjoint_impl(dp_plan *p, const void *J, const void *pi, const int16_t *u0_dev, void *scratch,
                        double *grad_dev, double *dgrade_dev, double *dspat_dev, void *stream)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (!(p->flags & DP_STORE_ALL_V)) return fail(DP_ESTATE, "adjoint needs a plan built with DP_STORE_ALL_V");
    if (!p->solved) return fail(DP_ESTATE, "adjoint before dp_solve");
    if (!J || !pi || !u0_dev || !scratch || !grad_dev) return fail(DP_EINVAL, "NULL buffer");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    size_t dgrade_off = 0, dspat_off = 0;
    for (size_t b = 0; b < p->inst.size(); b++) {
        const Inst &I = p->inst[b];
        double *gstage = dgrade_dev ? (double *)((char *)scratch + p->scr_gstage) : nullptr;
        double *gspat = dspat_dev && I.n_lights > 0 ? (double *)((char *)scratch + p->scr_gspat) : nullptr;
        double *rho_a = (double *)((char *)scratch + I.scr_rho);
        double *rho_b = rho_a + I.S;
        double *g = grad_dev + 5 * b;
        const float *Jb = (const float *)((const char *)J + I.J_off);
        const int16_t *pib = (const int16_t *)((const char *)pi + I.pi_off);
        double *gpart = (double *)((char *)scratch + p->scr_gpart);
        // both occupancy buffers start at zero; each stage zeroes the one it reads
        if (launch_fill_f64(g, 5, 0.0, s) || launch_fill_f64(rho_a, 2L * (long)I.S, 0.0, s) ||
            launch_fill_f64(gpart, 5L * 1024, 0.0, s) ||
            (gstage && launch_fill_f64(gstage, (long)adjoint_grade_slots(), 0.0, s)) ||
            (gspat && launch_fill_f64(gspat, 2L * (long)adjoint_grade_slots() * I.n_lights, 0.0, s)))
            return hip_fail(hipGetLastError(), "fill launch");
        if (launch_adjoint_root(I.P, Jb + I.S, u0_dev + b, rho_a, g, gstage, s))
            return hip_fail(hipGetLastError(), "adjoint root launch");
        for (int k = 1; k < I.N; k++) {
            const int L = I.light_of_stage[k];
            const TLEntry *tl = L >= 0 ? p->dev_tl + I.tl_dev_off + (size_t)L * I.P.n_t : nullptr;
            void *tab = (char *)scratch + p->scr_adjtab;
            if ((k == 1 || !I.same_tables[k - 1]) && launch_adjoint_table(I.P, k, tab, s))
                return hip_fail(hipGetLastError(), "adjoint table launch");
            double *gspat_L = gspat && L >= 0 ? gspat + 2 * adjoint_grade_slots() * (size_t)L : nullptr;
            if (launch_adjoint_stage(I.P, k, Jb + (size_t)(k + 1) * I.S, pib + (size_t)k * I.S, tl, tab, rho_a, rho_b,
                                     gpart, gstage, gspat_L, (p->flags & DP_ADJOINT_WIDE) != 0, s))
                return hip_fail(hipGetLastError(), "adjoint stage launch");
            double *t = rho_a;
            rho_a = rho_b;
            rho_b = t;
        }
        if (launch_adjoint_terminal(I.P, Jb + (size_t)I.N * I.S, rho_a, gpart, s))
            return hip_fail(hipGetLastError(), "adjoint terminal launch");
        if (launch_adjoint_reduce(gpart, g, s)) return hip_fail(hipGetLastError(), "adjoint reduce launch");
        if (gstage && launch_adjoint_grade(I.P, gstage, g, dgrade_dev + dgrade_off, s))
            return hip_fail(hipGetLastError(), "adjoint grade launch");
        if (gspat && launch_adjoint_spat(I.n_lights, gspat, g, dspat_dev + dspat_off, s))
            return hip_fail(hipGetLastError(), "adjoint signal-timing launch");
        dgrade_off += (size_t)I.N;
        dspat_off += 3 * (size_t)I.n_lights;
    }
    return DP_OK;
}

int dp_adjoint(dp_plan *p, const void *J, const void *pi, const int16_t *u0_dev, void *scratch, double *grad_dev,
               void *stream)
{
    return adjoint_impl(p, J, pi, u0_dev, scratch, grad_dev, nullptr, nullptr, stream);
}

int dp_adjoint_grade(dp_plan *p, const void *J, const void *pi, const int16_t *u0_dev, void *scratch,
                     double *grad_dev, double *dgrade_dev, void *stream)
{
    if (!dgrade_dev) return fail(DP_EINVAL, "NULL grade-sensitivity buffer");
    return adjoint_impl(p, J, pi, u0_dev, scratch, grad_dev, dgrade_dev, nullptr, stream);
}

int dp_adjoint_spat(dp_plan *p, const void *J, const void *pi, const int16_t *u0_dev, void *scratch,
                    double *grad_dev, double *dspat_dev, void *stream)
{
    if (!dspat_dev) return fail(DP_EINVAL, "NULL signal-timing sensitivity buffer");
    return adjoint_impl(p, J, pi, u0_dev, scratch, grad_dev, nullptr, dspat_dev, stream);
}

int dp_executed_evaluations(dp_plan *p, int64_t *counts, void *stream)
{
    if (!p || !counts) return fail(DP_EINVAL, "NULL argument");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    std::vector<unsigned long long> h(p->inst.size());
    e = hipMemcpyAsync(h.data(), p->dev_count, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "evaluation counters");
    for (size_t b = 0; b < h.size(); b++) counts[b] = (int64_t)h[b];
    return DP_OK;
}

int dp_device_check(dp_plan *p, void *stream)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    int w = 0;
    e = hipMemcpyAsync(&w, p->dev_err, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "device error word");
    if (w == 0) return DP_OK;
    const int zero = 0;
    e = hipMemcpyAsync(p->dev_err, &zero, sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "device error word reset");
    return fail(DP_EDEVICE, "device error word 0x%x:%s%s%s", w,
                (w & kDevErrCellOffset) ? " a SoC cell offset did not fit its int8 record field;" : "",
                (w & kDevErrWait) ? " a persistent sweep gave up waiting for a stage;" : "",
                (w & kDevErrNegative) ? " a terminal value (device terminal_V) was negative;" : "");
}

int dp_sweep_time(dp_plan *p, double *ms, int32_t *launches)
{
    if (!p || !ms || !launches) return fail(DP_EINVAL, "NULL argument");
    if (!(p->flags & DP_TIMING)) return fail(DP_ESTATE, "plan built without DP_TIMING");
    double tot = 0.0;
    for (int q = 0; q + 1 < p->n_ev_used; q += 2) {
        hipError_t e = hipEventSynchronize(p->ev[q + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float t = 0.0f;
        e = hipEventElapsedTime(&t, p->ev[q], p->ev[q + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        tot += t;
    }
    *ms = tot;
    *launches = p->n_ev_used / 2;
    p->n_ev_used = 0;
    return DP_OK;
}

void dp_destroy(dp_plan *p)
{
    if (!p) return;
    (void)hipSetDevice(p->device);
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    drop_graph(p);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    for (int q = 0; q < dp_plan::kSide; q++) {
        if (p->side[q]) (void)hipStreamDestroy(p->side[q]);
        if (p->join[q]) (void)hipEventDestroy(p->join[q]);
    }
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->state_ev) {
        (void)hipEventSynchronize(p->state_ev);
        (void)hipEventDestroy(p->state_ev);
    }
    if (p->state_host) (void)hipHostFree(p->state_host);
    if (p->tstream) (void)hipStreamDestroy(p->tstream);
    if (p->tfork) (void)hipEventDestroy(p->tfork);
    if (p->tjoin) (void)hipEventDestroy(p->tjoin);
    if (p->dev_tables) (void)hipFree(p->dev_tables);
    if (p->dev_ptables) (void)hipFree(p->dev_ptables);
    if (p->dev_params) (void)hipFree(p->dev_params);
    delete p;
}

}  // extern "C"

namespace ecodp {

int api_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int build_window_plan(const dp_problem_desc &d, int H_min, const dp_options *opt, int device, dp_plan **out)
{
    t_window.on = true;
    t_window.h_min = H_min;
    const int rc = dp_build_problem(&d, 1, opt, device, out);
    t_window = WindowBuild();
    return rc;
}

float *plan_terminal(dp_plan *p) { return p ? const_cast<float *>(p->inst[0].P.terminal_V) : nullptr; }

int plan_set_window(dp_plan *p, const double *grade, const double *vmax, const double *cycle, const double *red,
                    const double *offset, const double *yellow, double t0_abs, double v0, double soc0, hipStream_t s)
{
    Inst &I = p->inst[0];
    const int N = I.N, nl = (int)I.l_cycle.size();
    if (nl != N - 1) return fail(DP_ESTATE, "not a window plan (%d signals on %d stages)", nl, N);
    if (!(std::isfinite(v0) && v0 >= 0.0 && std::isfinite(soc0) && soc0 >= I.P.s_lo && soc0 <= I.P.s_hi &&
          std::isfinite(t0_abs)))
        return fail(DP_EINVAL, "window: x0 outside the grid or not finite");
    for (int k = 0; k < N; k++)
        if (!std::isfinite(grade[k])) return fail(DP_EINVAL, "window: grade %d not finite", k);
    for (int k = 0; k <= N; k++)
        if (!(std::isfinite(vmax[k]) && vmax[k] >= 0.0)) return fail(DP_EINVAL, "window: speed limit %d", k);
    for (int L = 0; L < nl; L++)
        if (!(std::isfinite(cycle[L]) && cycle[L] > 0.0 && std::isfinite(red[L]) && red[L] >= 0.0 &&
              red[L] <= cycle[L] && std::isfinite(offset[L]) && std::isfinite(yellow[L]) && yellow[L] >= 0.0 &&
              yellow[L] <= cycle[L] - red[L] && (yellow[L] == 0.0 || I.P.amin < 0.0)))
            return fail(DP_EINVAL, "window: signal of stage %d", L + 1);
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    // the parameter block's per-stage arrays, in the layout of the build:
    // cos and sin of the grade angle [N], speed limits [N+1], cycle, red,
    // offset and yellow of every signal, three spare zeros
    const size_t n_dbl = 3 * (size_t)N + 1 + 4 * (size_t)nl + 3;
    const size_t tl_n = (size_t)nl * I.P.n_t;
    const size_t o_dbl = align_up(sizeof(DevInst), 256);
    const size_t o_tl = o_dbl + align_up(sizeof(double) * n_dbl, 256);
    int rc = state_staging(p, o_tl + sizeof(TLEntry) * (tl_n ? tl_n : 1));
    if (rc) return rc;
    char *h = (char *)p->state_host;
    double *dbl = (double *)(h + o_dbl);
    for (int k = 0; k < N; k++) {
        const double G = grade[k];
        dbl[k] = 1.0 / std::sqrt(1.0 + G * G);
        dbl[N + k] = G * dbl[k];
    }
    for (int k = 0; k <= N; k++) dbl[2 * N + k] = vmax[k];
    for (int L = 0; L < nl; L++) {
        dbl[3 * N + 1 + L] = cycle[L];
        dbl[3 * N + 1 + nl + L] = red[L];
        dbl[3 * N + 1 + 2 * nl + L] = offset[L];
        dbl[3 * N + 1 + 3 * nl + L] = yellow[L];
    }
    for (int q = 0; q < 3; q++) dbl[3 * N + 1 + 4 * nl + q] = 0.0;
    I.l_cycle.assign(cycle, cycle + nl);
    I.l_red.assign(red, red + nl);
    I.l_off.assign(offset, offset + nl);
    I.l_yel.assign(yellow, yellow + nl);
    I.P.v0 = v0;
    I.P.soc0 = soc0;
    I.P.t0_abs = t0_abs;
    std::memcpy(h, &I.P, sizeof(DevInst));
    TLEntry *htl = (TLEntry *)(h + o_tl);
    for (int L = 0; L < nl; L++)
        build_tl(cycle[L], red[L], offset[L], yellow[L], t0_abs, I.P.t_f, I.P.n_t, I.P.wt, htl + (size_t)L * I.P.n_t);
    e = hipMemcpyAsync(p->dev_insts, h, sizeof(DevInst), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(const_cast<double *>(I.P.cosa), dbl, sizeof(double) * n_dbl, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && tl_n)
        e = hipMemcpyAsync(p->dev_tl + I.tl_dev_off, htl, sizeof(TLEntry) * tl_n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(p->state_ev, s);
    if (e != hipSuccess) return hip_fail(e, "window upload");
    p->state_pending = true;
    p->solved = false;
    return DP_OK;
}

}  // namespace ecodp
