// Host side of the ecodp C ABI: validation, FP64 host preprocessing (grade
// trigonometry, speed limits, signal red masks and wait times, Eq. 5c / 8),
// buffer layout, and the enqueueing of the kernels on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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

struct Inst {
    DevInst P;                 // device pointers filled at build
    int N = 0;
    size_t S = 0;              // slab elements
    std::vector<int> light_of_stage;
    size_t J_off = 0, pi_off = 0, traj_off = 0;
    size_t scr_st = 0, scr_bat = 0, scr_rho = 0, scr_nf = 0, scr_batj = 0, scr_hdr = 0;
    int sweep = 0;             // 1 = simple per-node kernel, 2 = grouped LDS kernel
    int jt = 8;                // SoC rows per workgroup of the grouped kernel
    int nsplit = 1;            // workgroups sharing one (speed node, SoC tile), each a slice of the controls
    size_t scr_pv = 0, scr_pu = 0, scr_rec = 0, scr_q = 0;
    int grid = 0;              // persistent workgroups of the grouped sweep
    int H = 0;                 // bound on the SoC-cell shift of one step
    size_t tl_dev_off = 0;     // offset (entries) of this instance's TL table in the plan's TL array
    int64_t evals = 0;
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
    if (!(K[2] > 0 && K[3] > 0 && K[4] > 0 && K[5] > 0 && K[6] > 0 && K[9] > 0 && K[13] > 0 && K[10] < K[11]))
        return fail(DP_EINVAL, "instance %d: vehicle constants out of range", b);
    for (int q = 0; q < 6; q++)
        if (!finite(d.fuel[q])) return fail(DP_EINVAL, "instance %d: fuel[%d] not finite", b, q);
    if ((long)d.n_te * d.n_tm > 32767) return fail(DP_EUNSUPPORTED, "instance %d: more than 32767 controls", b);
    if (d.n_v > 32767 || d.n_soc > 32767) return fail(DP_EUNSUPPORTED, "instance %d: grid too large", b);
    if (d.n_t > 1024) return fail(DP_EUNSUPPORTED, "instance %d: n_t > 1024", b);
    if (d.flags & ~DP_WAIT_AT_RED) return fail(DP_EINVAL, "instance %d: unknown flags", b);
    return DP_OK;
}

double gstep(double lo, double hi, int n) { return n > 1 ? (hi - lo) / (n - 1) : 0.0; }

// Signal table of one light: per time node, the red flag and the wait to
// green (Eq. 5c) in index space; FP64 on the host.
void build_tl(const dp_problem_desc &d, int L, TLEntry *out)
{
    const double ht = gstep(0.0, d.t_f, d.n_t);
    const double C = d.light_cycle[L], R = d.light_red[L], O = d.light_offset[L];
    const double wt = d.theta[3];
    for (int m = 0; m < d.n_t; m++) {
        TLEntry e;
        std::memset(&e, 0, sizeof e);
        const double tm = 0.0 + m * ht;
        double ph = std::fmod(d.t0_abs + tm - O, C);
        if (ph < 0.0) ph += C;
        e.red = ph < R ? 1 : 0;
        e.wc = -1;
        if (e.red) {
            const double tau = R - ph;
            const double delta = tau / ht;
            const double fl = std::floor(delta);
            long c = m + (long)fl;
            double f = delta - fl;
            if (c > d.n_t - 2) {
                f += (double)(c - (d.n_t - 2));
                c = d.n_t - 2;
            }
            if (f <= 1.0) {
                e.wc = (int32_t)c;
                e.wf = f;
                e.tau = tau;
                e.wcost = (float)(wt * tau);
                e.wf32 = (float)f;
                e.wg32 = (float)(1.0 - f);
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
    for (int i = 1; i < P.n_v; i++) {
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

int dp_build_problem(const dp_problem_desc *desc, int32_t n_inst, const dp_options *opt, int device, dp_plan **out)
{
    if (!out) return fail(DP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!desc || n_inst < 1) return fail(DP_EINVAL, "need at least one problem description");
    if (opt && (opt->flags & ~(DP_STORE_ALL_V | DP_TIMING))) return fail(DP_EINVAL, "unknown option flags");
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
    std::vector<std::vector<double>> cosa(n_inst), sina(n_inst), vmax(n_inst), lc(n_inst), lr(n_inst), lo(n_inst);
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
        for (int L = 0; L < d.n_lights; L++) {
            I.light_of_stage[d.light_stage[L]] = L;
            lc[b].push_back(d.light_cycle[L]);
            lr[b].push_back(d.light_red[L]);
            lo[b].push_back(d.light_offset[L]);
        }
        param_bytes += align_up(sizeof(double) * (2 * N + (N + 1) + 3 * d.n_lights + 3), 256);
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
        dbl.resize(dbl.size() + 3, 0.0);
        const double *dd = (const double *)put(dbl.data(), sizeof(double) * dbl.size());
        P.cosa = dd;
        P.sina = dd + N;
        P.vmax = dd + 2 * N;
        const int nl = d.n_lights;
        P.l_cycle = dd + 3 * N + 1;
        P.l_red = P.l_cycle + nl;
        P.l_off = P.l_red + nl;
        P.light_of_stage = (const int *)put(I.light_of_stage.data(), sizeof(int) * (N + 1));
        P.terminal_V = d.terminal_V ? (const float *)put(d.terminal_V, sizeof(float) * I.S) : nullptr;
        for (int L = 0; L < nl; L++) build_tl(d, L, host_tl + I.tl_dev_off + (size_t)L * d.n_t);

        const int nst = (p->flags & DP_STORE_ALL_V) ? N + 1 : 2;
        I.J_off = J_off;
        J_off += align_up(sizeof(float) * I.S * nst, 256);
        I.pi_off = pi_off;
        pi_off += align_up(sizeof(int16_t) * I.S * N, 256);
        I.traj_off = traj_off;
        traj_off += (size_t)(N + 1) * 8;
        // state-sweep variant: the grouped LDS kernel when its tables and
        // staged planes fit, else the simple per-node kernel
        I.H = soc_shift_bound(P, d);
        // SoC rows per workgroup: the largest tile that still leaves about
        // three resident waves per SIMD (LDS of one CU is shared by its
        // workgroups); a caller tile overrides
        const size_t lds_cu = (size_t)p->lds_per_cu;
        const int waves = (d.n_t + 62) / 63;
        auto waves_per_simd = [&](int t) {
            const size_t bytes = lds_sweep_bytes(t, I.H, d.n_t);
            if (bytes > lds_cu) return 0.0;
            size_t wg = lds_cu / bytes;
            if (wg * waves > 32) wg = 32 / waves;
            return (double)(wg * waves) / 4.0;
        };
        int jt = 0;
        if (p->opt.tile[0] == 4 || p->opt.tile[0] == 8 || p->opt.tile[0] == 16) {
            jt = p->opt.tile[0];
        } else {
            const int cand[3] = {16, 8, 4};
            double best_w = 0.0;
            for (int t : cand) {
                if (t > 4 && d.n_soc < t) continue;
                const double w = waves_per_simd(t);
                if (w >= 2.75) {
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
        const bool lds_fits = lds_sweep_bytes(jt, I.H, d.n_t) <= lds_cu && d.n_t <= 1008 && P.n_u <= 1024 &&
                              d.n_v - 1 <= kSortBins;
        I.jt = jt;
        I.sweep = p->opt.kernel == 1 ? 1 : (lds_fits ? 2 : 1);
        if (p->opt.kernel == 2 && !lds_fits) {
            (void)hipFree(p->dev_params);
            delete p;
            return fail(DP_EUNSUPPORTED, "instance %d: grouped sweep does not fit (n_t %d, n_u %d, H %d)", b, d.n_t,
                        P.n_u, I.H);
        }
        if (lds_fits) {
            size_t wg = lds_cu / lds_sweep_bytes(jt, I.H, d.n_t);
            if (wg * waves > 32) wg = 32 / waves;
            if (wg < 1) wg = 1;
            I.grid = (int)(wg * (size_t)p->n_cu);
        }
        I.scr_st = scr;
        scr += align_up(sizeof(SortedEntry) * d.n_v * P.n_u, 256);
        I.scr_nf = scr;
        scr += align_up(sizeof(int) * d.n_v, 256);
        I.scr_bat = scr;   // BatEntry (simple kernel) or float2 weights (grouped kernel)
        scr += align_up(sizeof(BatEntry) * ((size_t)d.n_v * P.n_u * d.n_soc + 16), 256);
        if (I.sweep == 2) {
            const size_t ntiles = (d.n_soc + I.jt - 1) / I.jt;
            // enough workgroups for 256 CUs: split the control list when the
            // (speed node, SoC tile) grid alone is small
            const long base_wg = (long)d.n_v * (long)ntiles;
            int ns = (int)((2048 + base_wg - 1) / base_wg);
            if (p->opt.tile[1] > 0) ns = p->opt.tile[1];
            if (ns > 16) ns = 16;
            if (ns > P.n_u) ns = P.n_u;
            if (ns < 1) ns = 1;
            I.nsplit = ns;
            if (ns > 1) {
                I.scr_pv = scr;
                scr += align_up(sizeof(float) * I.S * ns, 256);
                I.scr_pu = scr;
                scr += align_up(sizeof(int16_t) * I.S * ns, 256);
            }
            I.scr_q = scr;
            scr += align_up(sizeof(int) * 8 * (size_t)N, 256);
            I.scr_rec = scr;
            scr += align_up(sizeof(float) * (size_t)d.n_v * ntiles * P.n_u * (12 + 2 * I.jt), 256);
            I.scr_batj = scr;
            scr += align_up(sizeof(int) * ((size_t)d.n_v * P.n_u * d.n_soc + 16), 256);
            I.scr_hdr = scr;
            scr += align_up(sizeof(int) * ((size_t)d.n_v * P.n_u * ntiles + 16), 256);
        }
        I.scr_rho = scr;
        scr += align_up(sizeof(double) * I.S * 2, 256);
        I.evals = (int64_t)N * (int64_t)I.S * P.n_u;
    }
    p->bytes_J = J_off;
    p->bytes_pi = pi_off;
    p->bytes_scratch = scr;
    if ((e = hipMemcpy(p->dev_params, host.data(), host.size(), hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(p->dev_params);
        delete p;
        return hip_fail(e, "parameter upload");
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
    return DP_OK;
}

static float *slab_ptr(dp_plan *p, const Inst &I, void *J, int k)
{
    const int idx = (p->flags & DP_STORE_ALL_V) ? k : (k & 1);
    return (float *)((char *)J + I.J_off) + (size_t)idx * I.S;
}

static int enqueue_stage(dp_plan *p, const Inst &I, int k, const float *Jn, float *Jk, int16_t *pik, void *scratch,
                         hipStream_t s, bool zero_queue)
{
    StageEntry *st = (StageEntry *)((char *)scratch + I.scr_st);
    SortedEntry *sst = (SortedEntry *)((char *)scratch + I.scr_st);
    int *nfeas = (int *)((char *)scratch + I.scr_nf);
    BatEntry *bat = (BatEntry *)((char *)scratch + I.scr_bat);
    const int L = I.light_of_stage[k];
    const TLEntry *tl = L >= 0 ? p->dev_tl + I.tl_dev_off + (size_t)L * I.P.n_t : nullptr;
    float2 *batw = (float2 *)((char *)scratch + I.scr_bat);
    int *batj = (int *)((char *)scratch + I.scr_batj);
    int *hdr = (int *)((char *)scratch + I.scr_hdr);
    if (I.sweep == 2) {
        if (zero_queue && launch_fill_i32((int *)((char *)scratch + I.scr_q) + 8 * k, 8, 0, s))
            return hip_fail(hipGetLastError(), "queue reset launch");
        if (launch_stage_sorted(I.P, k, I.jt, sst, nfeas, batw, batj, hdr, (float *)((char *)scratch + I.scr_rec), s))
            return hip_fail(hipGetLastError(), "stage table launch");
    } else {
        if (launch_stage_table(I.P, k, st, bat, s)) return hip_fail(hipGetLastError(), "stage table launch");
    }
    const bool timing = (p->flags & DP_TIMING) != 0;
    if (timing) {
        if (p->n_ev_used + 2 > (int)p->ev.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
                return fail(DP_EDEVICE, "event creation failed");
            p->ev.push_back(a);
            p->ev.push_back(b);
        }
        (void)hipEventRecord(p->ev[p->n_ev_used], s);
    }
    float *part_v = (float *)((char *)scratch + I.scr_pv);
    int16_t *part_u = (int16_t *)((char *)scratch + I.scr_pu);
    int *queue = (int *)((char *)scratch + I.scr_q) + 8 * k;
    const int rc = I.sweep == 2 ? launch_sweep_lds(I.jt, I.P, k, Jn, Jk, pik, nfeas,
                                                   (const float *)((char *)scratch + I.scr_rec), batj, tl, I.H,
                                                   I.nsplit, part_v, part_u, queue, I.grid, s)
                                : launch_sweep(I.P, k, Jn, Jk, pik, st, bat, tl, s);
    if (rc) return hip_fail(hipGetLastError(), "sweep launch");
    if (timing) {
        (void)hipEventRecord(p->ev[p->n_ev_used + 1], s);
        p->n_ev_used += 2;
    }
    return DP_OK;
}

int dp_solve(dp_plan *p, void *J, void *pi, void *scratch, float *V0_dev, int16_t *u0_dev, void *stream)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (!J || !pi || !scratch || !V0_dev || !u0_dev) return fail(DP_EINVAL, "NULL buffer");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    for (size_t b = 0; b < p->inst.size(); b++) {
        const Inst &I = p->inst[b];
        if (launch_terminal(I.P, slab_ptr(p, I, J, I.N), s)) return hip_fail(hipGetLastError(), "terminal launch");
        if (I.sweep == 2 && launch_fill_i32((int *)((char *)scratch + I.scr_q), 8L * I.N, 0, s))
            return hip_fail(hipGetLastError(), "queue reset launch");
        for (int k = I.N - 1; k >= 0; k--) {
            int16_t *pik = (int16_t *)((char *)pi + I.pi_off) + (size_t)k * I.S;
            int rc = enqueue_stage(p, I, k, slab_ptr(p, I, J, k + 1), slab_ptr(p, I, J, k), pik, scratch, s, false);
            if (rc) return rc;
        }
        if (launch_root(I.P, slab_ptr(p, I, J, 1), V0_dev + b, u0_dev + b, s))
            return hip_fail(hipGetLastError(), "root launch");
    }
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
    return enqueue_stage(p, I, k, J_next, J_out, pi_out, scratch, (hipStream_t)stream, true);
}

int dp_rollout(dp_plan *p, const void *pi, const int16_t *u0_dev, double *traj_dev, int32_t *status_dev, void *stream)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (!pi || !u0_dev || !traj_dev || !status_dev) return fail(DP_EINVAL, "NULL buffer");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    for (size_t b = 0; b < p->inst.size(); b++) {
        const Inst &I = p->inst[b];
        const int16_t *pib = (const int16_t *)((const char *)pi + I.pi_off);
        if (launch_rollout(I.P, pib, u0_dev + b, nullptr, traj_dev + I.traj_off, status_dev + 2 * b, s))
            return hip_fail(hipGetLastError(), "rollout launch");
    }
    return DP_OK;
}

int dp_adjoint(dp_plan *p, const void *J, const void *pi, const int16_t *u0_dev, void *scratch, double *grad_dev,
               void *stream)
{
    if (!p) return fail(DP_EINVAL, "plan is NULL");
    if (!(p->flags & DP_STORE_ALL_V)) return fail(DP_ESTATE, "adjoint needs a plan built with DP_STORE_ALL_V");
    if (!p->solved) return fail(DP_ESTATE, "adjoint before dp_solve");
    if (!J || !pi || !u0_dev || !scratch || !grad_dev) return fail(DP_EINVAL, "NULL buffer");
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    for (size_t b = 0; b < p->inst.size(); b++) {
        const Inst &I = p->inst[b];
        double *rho_a = (double *)((char *)scratch + I.scr_rho);
        double *rho_b = rho_a + I.S;
        double *g = grad_dev + 5 * b;
        const float *Jb = (const float *)((const char *)J + I.J_off);
        const int16_t *pib = (const int16_t *)((const char *)pi + I.pi_off);
        if (launch_fill_f64(g, 5, 0.0, s) || launch_fill_f64(rho_a, (long)I.S, 0.0, s))
            return hip_fail(hipGetLastError(), "fill launch");
        if (launch_adjoint_root(I.P, Jb + I.S, u0_dev + b, rho_a, g, s))
            return hip_fail(hipGetLastError(), "adjoint root launch");
        for (int k = 1; k < I.N; k++) {
            const int L = I.light_of_stage[k];
            const TLEntry *tl = L >= 0 ? p->dev_tl + I.tl_dev_off + (size_t)L * I.P.n_t : nullptr;
            if (launch_fill_f64(rho_b, (long)I.S, 0.0, s)) return hip_fail(hipGetLastError(), "fill launch");
            if (launch_adjoint_stage(I.P, k, Jb + (size_t)(k + 1) * I.S, pib + (size_t)k * I.S, tl, rho_a, rho_b, g, s))
                return hip_fail(hipGetLastError(), "adjoint stage launch");
            double *t = rho_a;
            rho_a = rho_b;
            rho_b = t;
        }
        if (launch_adjoint_terminal(I.P, Jb + (size_t)I.N * I.S, rho_a, g, s))
            return hip_fail(hipGetLastError(), "adjoint terminal launch");
    }
    return DP_OK;
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
    if (p->dev_params) (void)hipFree(p->dev_params);
    delete p;
}

}  // extern "C"
