// HIP kernels (gfx950) of the eco-driving DP: terminal slab (Eq. 9a), stage
// table (Sec. IV "Kernel 1": per speed node and control), state sweep
// (Sec. IV "Kernel 2": per state node, minimum over controls, Eq. 9b-d),
// exact root step at x0 (Eq. 6).
#include "dp_internal.h"

namespace ecodp {

// ---------------------------------------------------------------- terminal --

// J_N = min(J_inf, w_soc (xi_j - xi_ref)^2 + terminal_V) in FP64, one FP32
// rounding; nodes above the stage-N speed limit take J_inf.  A negative
// terminal_V value (the sweep's minimum assumes non-negative costs) sets
// kDevErrNegative in the device error word.
__global__ void k_terminal_jobs(const DevInst *__restrict__ insts, char *__restrict__ J,
                                const long long *__restrict__ jN_off, int *__restrict__ err)
{
#pragma clang fp contract(off)
    const DevInst &P = insts[blockIdx.y];
    float *__restrict__ JN = (float *)(J + jN_off[blockIdx.y]);
    const long S = (long)P.n_v * P.n_s * P.n_t;
    for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < S; n += (long)gridDim.x * blockDim.x) {
        const int m = (int)(n % P.n_t);
        const long ij = n / P.n_t;
        const int j = (int)(ij % P.n_s);
        const int i = (int)(ij / P.n_s);
        (void)m;
        const double v = P.v_lo + i * P.hv;
        const double xi = P.s_lo + j * P.hs;
        double val = P.wsoc * (xi - P.xiref) * (xi - P.xiref);
        if (P.terminal_V) {
            const float tv = P.terminal_V[n];
            if (tv < 0.0f) atomicOr(err, kDevErrNegative);
            val += (double)tv;
        }
        if (v > P.vmax[P.N] || !(val < P.Jinf)) val = P.Jinf;
        JN[n] = (float)val;
    }
}

// Terminal table of a horizon starting at clock t_shift of a longer solve
// (Sec. III after Eq. 9): per node, the linear interpolation in time of that
// solve's value slab, FP64 with one FP32 rounding, capped at J_inf.
__global__ void k_terminal_shift(const float *__restrict__ src, long nvs, int n_src, double h_src, double t_shift,
                                 int n_dst, double h_dst, double Jinf, float *__restrict__ dst)
{
#pragma clang fp contract(off)
    const long S = nvs * n_dst;
    for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < S; n += (long)gridDim.x * blockDim.x) {
        const int m = (int)(n % n_dst);
        const long ij = n / n_dst;
        const double t = t_shift + m * h_dst;
        const double r = t / h_src;
        double val = Jinf;
        if (r <= (double)(n_src - 1)) {
            int c = (int)floor(r);
            if (c > n_src - 2) c = n_src - 2;
            const double f = r - c;
            const float *row = src + ij * n_src;
            val = (1.0 - f) * (double)row[c] + f * (double)row[c + 1];
            if (!(val < Jinf)) val = Jinf;
        }
        dst[n] = (float)val;
    }
}

int launch_terminal_shift(const float *src, long nvs, int n_src, double h_src, double t_shift, int n_dst, double h_dst,
                          double Jinf, float *dst, hipStream_t s)
{
    long blocks = (nvs * n_dst + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_terminal_shift, dim3((unsigned)blocks), dim3(256), 0, s, src, nvs, n_src, h_src, t_shift,
                       n_dst, h_dst, Jinf, dst);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------- stage table --

// One thread per (speed node i, control u, SoC node j), j fastest.  The
// powertrain part (speed and time coordinates, stage cost) is written once
// per (i, u) by the j == 0 thread; every thread writes its battery coordinate.
__global__ void k_stage_table(DevInst P, int k, StageEntry *__restrict__ st, BatEntry *__restrict__ bat,
                              unsigned long long *__restrict__ count)
{
#pragma clang fp contract(off)
    const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long total = (long)P.n_v * P.n_u * P.n_s;
    if (idx >= total) return;
    const int j = (int)(idx % P.n_s);
    const long iu = idx / P.n_s;
    const int u = (int)(iu % P.n_u);
    const int i = (int)(iu / P.n_u);
    const double v = P.v_lo + i * P.hv;
    const PT p = powertrain(P, k, v, u / P.n_m, u % P.n_m);
    bool ok = p.st == 0;
    int iv = 0, dtc = 0;
    double fv = 0.0, ft = 0.0;
    if (ok) {
        const double rv = (p.v1 - P.v_lo) / P.hv;
        if (!(rv >= 0.0 && rv <= P.n_v - 1)) ok = false;
        else cell_of(rv, P.n_v, iv, fv);
        const double delta = p.dt / P.ht;
        if (!(delta < P.n_t)) {
            ok = false;
        } else {
            const double fl = floor(delta);
            dtc = (int)fl;
            ft = delta - fl;
        }
    }
    // the simple sweep evaluates every node of a feasible pair (speed node
    // under the stage's limit) and skips the others: count those evaluations
    const unsigned long long counted = __ballot(j == 0 && ok && !(v > P.vmax[k]));
    if ((threadIdx.x & 63) == 0 && counted)
        atomicAdd(count, (unsigned long long)__popcll(counted) * (unsigned long long)P.n_s * P.n_t);
    if (j == 0) {
        StageEntry e;
        e.c = (float)p.cost;
        e.fv = (float)fv;
        e.gv = (float)(1.0 - fv);
        e.ft = (float)ft;
        e.gt = (float)(1.0 - ft);
        e.iv = ok ? (int16_t)iv : (int16_t)-1;
        e.dtc = (int16_t)dtc;
        st[iu] = e;
    }
    BatEntry b;
    b.jx = -1;
    b.fx = 0.0f;
    b.gx = 0.0f;
    if (ok) {
        double I;
        const double xi = P.s_lo + j * P.hs;
        if (battery_current(P, p.Pb, xi, I)) {
            const double rs = (double)j - (p.dt * I) / (P.Cnom * P.hs);
            if (rs >= 0.0 && rs <= P.n_s - 1) {
                int jx;
                double fx;
                cell_of(rs, P.n_s, jx, fx);
                b.jx = jx;
                b.fx = (float)fx;
                b.gx = (float)(1.0 - fx);
            }
        }
    }
    bat[idx] = b;
}

// ------------------------------------------------------------- state sweep --

// One workgroup per (speed node i, tile of JT SoC nodes); one lane per time
// node m.  For every control (wave-uniform loop, ascending u) and every SoC
// node of the tile: Q = c + trilinear J_{k+1} at the successor, kept if
// strictly below the running minimum (initially J_inf), so the lowest u wins a
// tie.  Signal nodes where the vehicle has to stop (red, or yellow past its
// braking distance) are overridden at the store: J_inf for a moving vehicle,
// the wait value (Eq. 5c) for the zero-speed row.
template <int JT>
__global__ void __launch_bounds__(1024) k_sweep_naive(DevInst P, int k, const float *__restrict__ Jn,
                                                      float *__restrict__ Jk, int16_t *__restrict__ pik,
                                                      const StageEntry *__restrict__ st,
                                                      const BatEntry *__restrict__ bat,
                                                      const TLEntry *__restrict__ tl)
{
    const int i = blockIdx.y;
    const int j0 = blockIdx.x * JT;
    const int m = threadIdx.x;
    const int nt = P.n_t, ns = P.n_s;
    const long SV = (long)ns * nt;
    const float Jinf = (float)P.Jinf;
    float best[JT];
    int bu[JT];
#pragma unroll
    for (int q = 0; q < JT; q++) {
        best[q] = Jinf;
        bu[q] = -1;
    }
    double v;
    {
#pragma clang fp contract(off)
        v = P.v_lo + i * P.hv;
    }
    const bool row_ok = !(v > P.vmax[k]);
    if (row_ok) {
        const StageEntry *sti = st + (long)i * P.n_u;
        const BatEntry *bti = bat + (long)i * P.n_u * ns;
        for (int u = 0; u < P.n_u; u++) {
            const StageEntry e = sti[u];
            if (e.iv < 0) continue;
            int tc = m + e.dtc;
            float ft = e.ft, gt = e.gt;
            bool ok = m < nt;
            if (tc > nt - 2) {
                if (tc == nt - 1 && ft == 0.0f) {
                    tc = nt - 2;
                    ft = 1.0f;
                    gt = 0.0f;
                } else {
                    ok = false;
                }
            }
            if (!ok) tc = 0;
            const float *pv = Jn + (long)e.iv * SV + tc;
#pragma unroll
            for (int q = 0; q < JT; q++) {
                const int j = j0 + q;
                if (j >= ns) break;
                const BatEntry b = bti[(long)u * ns + j];
                if (b.jx < 0) continue;
                const float *p0 = pv + (long)b.jx * nt;
                const float a00 = gt * p0[0] + ft * p0[1];
                const float a01 = gt * p0[nt] + ft * p0[nt + 1];
                const float a10 = gt * p0[SV] + ft * p0[SV + 1];
                const float a11 = gt * p0[SV + nt] + ft * p0[SV + nt + 1];
                const float b0 = b.gx * a00 + b.fx * a01;
                const float b1 = b.gx * a10 + b.fx * a11;
                const float Q = e.c + (e.gv * b0 + e.fv * b1);
                if (ok && Q < best[q]) {
                    best[q] = Q;
                    bu[q] = u;
                }
            }
        }
    }
    if (m >= nt) return;
    TLEntry t;
    const bool has_tl = tl != nullptr;
    if (has_tl) t = tl[m];
    const bool stop = has_tl && tl_stop(t, v, P.amin);
#pragma unroll
    for (int q = 0; q < JT; q++) {
        const int j = j0 + q;
        if (j >= ns) break;
        float J = best[q];
        int pu = bu[q];
        if (stop) {
            J = Jinf;
            pu = -1;
            if (i == P.zero_row && P.wait && t.wc >= 0) {
                const float *pw = Jn + ((long)i * ns + j) * nt + t.wc;
                const float w = wait_value(t, pw);
                if (w < Jinf) {
                    J = w;
                    pu = -2;
                }
            }
        }
        const long n = ((long)i * ns + j) * nt + m;
        Jk[n] = J;
        pik[n] = (int16_t)pu;
    }
}

// -------------------------------------------------------------------- root --

// Eq. 6 at the actual state x0 = (v0, soc0, t = 0): every control in FP64
// coordinates and an FP32 value, then a lexicographic (value, u) minimum over
// the workgroup.
// The parameter block comes from device memory, so that a recorded solve
// picks up a state moved by dp_set_state.
__device__ void root_one(const DevInst &P, const float *__restrict__ J1, float *V0, int16_t *u0)
{
#pragma clang fp contract(off)
    __shared__ float sv[256];
    __shared__ int su[256];
    const float Jinf = (float)P.Jinf;
    float best = Jinf;
    int bu = -1;
    const int nt = P.n_t, ns = P.n_s;
    const long SV = (long)ns * nt;
    if (!(P.v0 > P.vmax[0])) {
        const double rs0 = (P.soc0 - P.s_lo) / P.hs;
        for (int u = threadIdx.x; u < P.n_u; u += blockDim.x) {
            const PT p = powertrain(P, 0, P.v0, u / P.n_m, u % P.n_m);
            if (p.st) continue;
            double I;
            if (!battery_current(P, p.Pb, P.soc0, I)) continue;
            const double rv = (p.v1 - P.v_lo) / P.hv;
            if (!(rv >= 0.0 && rv <= P.n_v - 1)) continue;
            const double rs = rs0 - (p.dt * I) / (P.Cnom * P.hs);
            if (!(rs >= 0.0 && rs <= P.n_s - 1)) continue;
            const double delta = p.dt / P.ht;
            if (!(delta <= P.n_t - 1)) continue;
            int iv, jx, tc;
            double fv, fx, ft;
            cell_of(rv, P.n_v, iv, fv);
            cell_of(rs, P.n_s, jx, fx);
            cell_of(delta, P.n_t, tc, ft);
            const float gt = (float)(1.0 - ft), ftf = (float)ft;
            const float gx = (float)(1.0 - fx), fxf = (float)fx;
            const float gv = (float)(1.0 - fv), fvf = (float)fv;
            const float *p0 = J1 + (long)iv * SV + (long)jx * nt + tc;
            const float a00 = gt * p0[0] + ftf * p0[1];
            const float a01 = gt * p0[nt] + ftf * p0[nt + 1];
            const float a10 = gt * p0[SV] + ftf * p0[SV + 1];
            const float a11 = gt * p0[SV + nt] + ftf * p0[SV + nt + 1];
            const float b0 = gx * a00 + fxf * a01;
            const float b1 = gx * a10 + fxf * a11;
            const float Q = (float)p.cost + (gv * b0 + fvf * b1);
            if (Q < best) {
                best = Q;
                bu = u;
            }
        }
    }
    sv[threadIdx.x] = best;
    su[threadIdx.x] = bu;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const float ov = sv[threadIdx.x + s];
            const int ou = su[threadIdx.x + s];
            const float mv = sv[threadIdx.x];
            const int mu = su[threadIdx.x];
            if (ov < mv || (ov == mv && ou >= 0 && (mu < 0 || ou < mu))) {
                sv[threadIdx.x] = ov;
                su[threadIdx.x] = ou;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *V0 = sv[0];
        *u0 = (int16_t)su[0];
    }
}

// Every instance's root step in one launch, one workgroup per instance; J_1
// of instance b at byte offset j1_off[b] from J.
__global__ void __launch_bounds__(256) k_root_jobs(const DevInst *__restrict__ insts, const char *__restrict__ J,
                                                   const long long *__restrict__ j1_off, float *V0, int16_t *u0)
{
    const int b = blockIdx.x;
    root_one(insts[b], (const float *)(J + j1_off[b]), V0 + b, u0 + b);
}

// ------------------------------------------------------------------ launch --

int launch_terminal_jobs(const DevInst *insts, int n_inst, long max_slab, void *J, const long long *jN_off,
                         int *err, hipStream_t s)
{
    long blocks = (max_slab + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_terminal_jobs, dim3((unsigned)blocks, n_inst), dim3(256), 0, s, insts, (char *)J, jN_off, err);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_stage_table(const DevInst &P, int k, StageEntry *st, BatEntry *bat, unsigned long long *count,
                       hipStream_t s)
{
    const long total = (long)P.n_v * P.n_u * P.n_s;
    const int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_stage_table, dim3(blocks), dim3(256), 0, s, P, k, st, bat, count);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sweep(const DevInst &P, int k, const float *Jn, float *Jk, int16_t *pik, const StageEntry *st,
                 const BatEntry *bat, const TLEntry *tl, hipStream_t s)
{
    constexpr int JT = 4;
    const int threads = ((P.n_t + 63) / 64) * 64;
    dim3 grid((P.n_s + JT - 1) / JT, P.n_v);
    hipLaunchKernelGGL(k_sweep_naive<JT>, grid, dim3(threads), 0, s, P, k, Jn, Jk, pik, st, bat, tl);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_root_jobs(const DevInst *insts, int n_inst, const void *J, const long long *j1_off, float *V0, int16_t *u0,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_root_jobs, dim3(n_inst), dim3(256), 0, s, insts, (const char *)J, j1_off, V0, u0);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ecodp
