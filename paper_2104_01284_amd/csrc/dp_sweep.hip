// Grouped, LDS-staged state sweep (Sec. IV "Kernel 2") for gfx950.
//
// For a fixed output speed node i and control u every interpolation weight
// and every cell offset is the same for all time nodes (the time coordinate
// advances by the same dt/h_t from every node) and the same for all time
// nodes of one SoC node.  The sweep therefore runs lanes over time nodes with
// a wave-uniform control loop, and
//  * visits the controls of node i grouped by their successor's lower speed
//    cell iv (ascending, controls ascending inside a group), so the two
//    next-stage speed planes iv, iv+1 (the SoC rows of the tile plus a halo,
//    all times) are staged into LDS once per group;
//  * interpolates in speed first (V), then in time with the neighbouring
//    lane's V obtained by a DPP wave shift (one LDS read per plane and time),
//    and shares each (speed, time) bilinear row T between the two SoC nodes
//    whose SoC cell it bounds;
//  * keeps the running minimum and argmin of a tile of SoC nodes in registers.
// A wave covers 63 consecutive time nodes; its lane 63 only supplies the time
// neighbour of lane 62.  Exact FP32 ties keep the first control visited.
#include "dp_internal.h"

namespace ecodp {

// ------------------------------------------------------- sorted stage table --

// One workgroup per (job, speed node i), one thread per control: the FP64
// powertrain model (as the per-pair stage table) and a stable counting sort
// of the feasible controls by successor speed cell.
__global__ void __launch_bounds__(1024) k_stage_sort(StageBase B)
{
    __shared__ int s_hist[kSortBins];
    __shared__ int s_min, s_max, s_cnt;
    const StageJob &jb = B.jobs[blockIdx.y];
    const DevInst &P = B.insts[jb.inst];
    const int k = jb.k;
    const int i = blockIdx.x;
    if (i >= P.n_v) return;
    SortedEntry *__restrict__ out = (SortedEntry *)(B.scr + jb.st);
    double2 *__restrict__ pw = (double2 *)(B.scr + jb.pw);
    int *__restrict__ nfeas = (int *)(B.scr + jb.nf);
    const int u = threadIdx.x;
    const int nu = P.n_u;
    if (u == 0) {
        s_min = 0x7fffffff;
        s_max = -1;
        s_cnt = 0;
    }
    for (int q = threadIdx.x; q < kSortBins; q += blockDim.x) s_hist[q] = 0;
    __syncthreads();
    SortedEntry e;
    double2 pbdt = make_double2(0.0, 0.0);   // battery power and time step, for the battery records
    int iv = -1;
    if (u < nu) {
#pragma clang fp contract(off)
        const double v = P.v_lo + i * P.hv;
        const PT p = powertrain(P, k, v, u / P.n_m, u % P.n_m);
        bool ok = p.st == 0;
        int c = 0, dtc = 0;
        double fv = 0.0, ft = 0.0;
        if (ok) {
            const double rv = (p.v1 - P.v_lo) / P.hv;
            if (!(rv >= 0.0 && rv <= P.n_v - 1)) ok = false;
            else cell_of(rv, P.n_v, c, fv);
            const double delta = p.dt / P.ht;
            if (!(delta < P.n_t)) {
                ok = false;
            } else {
                const double fl = floor(delta);
                dtc = (int)fl;
                ft = delta - fl;
            }
        }
        e.c = (float)p.cost;
        e.fv = (float)fv;
        e.gv = (float)(1.0 - fv);
        e.ft = (float)ft;
        e.rt = (float)(ft / (1.0 - ft));   // ft < 1, so finite
        e.iv = c;
        e.dtc = dtc;
        e.u = u;
        pbdt = make_double2(p.Pb, p.dt);
        if (ok) iv = c;
    }
    if (iv >= 0) {
        atomicMin(&s_min, iv);
        atomicMax(&s_max, iv);
        atomicAdd(&s_cnt, 1);
    }
    __syncthreads();
    if (s_cnt == 0) {
        if (threadIdx.x == 0) nfeas[i] = 0;
        return;
    }
    const int base = s_min;
    if (iv >= 0) atomicAdd(&s_hist[iv - base], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        const int bins = s_max - s_min + 1;
        for (int q = 0; q < bins; q++) {
            const int c = s_hist[q];
            s_hist[q] = run;
            run += c;
        }
        nfeas[i] = s_cnt;
    }
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    for (int ww = 0; ww < nw; ww++) {
        if (w == ww) {
            const unsigned long long active = __ballot(iv >= 0);
            unsigned long long rem = active;
            int rank = 0, cnt = 0;
            while (rem) {
                const int leader = __ffsll((long long)rem) - 1;
                const int val = __builtin_amdgcn_readlane(iv, leader);
                const unsigned long long msk = __ballot(iv == val) & active;
                if (iv == val) {
                    rank = __popcll(msk & __lanemask_lt());
                    cnt = __popcll(msk);
                }
                rem &= ~msk;
            }
            if (iv >= 0) {
                const int pos = s_hist[iv - base] + rank;
                out[(long)i * nu + pos] = e;
                pw[(long)i * nu + pos] = pbdt;
                if (rank == cnt - 1) s_hist[iv - base] += cnt;
            }
        }
        __syncthreads();
    }
}

// Speed nodes of a job in decreasing order of the work they carry (feasible
// controls; none above the stage's speed limit), ties by node index, so
// that the sweep hands out its longest items first.
__global__ void __launch_bounds__(256) k_stage_rank(StageBase B)
{
    const StageJob &jb = B.jobs[blockIdx.x];
    const DevInst &P = B.insts[jb.inst];
    const int *__restrict__ nfeas = (const int *)(B.scr + jb.nf);
    int *__restrict__ order = (int *)(B.scr + jb.nf) + P.n_v;
    const int nv = P.n_v, k = jb.k;
    auto work = [&](int i) {
        double v;
        {
#pragma clang fp contract(off)
            v = P.v_lo + i * P.hv;
        }
        return v > P.vmax[k] ? 0 : nfeas[i];
    };
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        const int w = work(i);
        int rank = 0;
        for (int o = 0; o < nv; o++) {
            const int wo = work(o);
            rank += (wo > w || (wo == w && o < i)) ? 1 : 0;
        }
        order[rank] = i;
    }
}

// Dwords of one packed record: first the SoC weights of the tile's rows, for
// each group of R = min(JT, 8) rows the R lower-cell weights gx gt then the R
// upper-cell weights fx gt (a wave reads its group's 2R weights with one LDS
// load, lane l taking weight l mod 2R, and broadcasts weight q to all lanes
// with DPP row_newbcast); then 8 scalars: c, fv, gv, rt, ft, iv | dtc << 16,
// u | hdr << 16 and one spare (read the same way, lane l taking scalar l); then
// the SoC cells of the tile's rows as int8 offsets from the row (JT / 4
// dwords).
__host__ __device__ constexpr int rec_scalars(int JT) { return 2 * JT; }
__host__ __device__ constexpr int rec_cells(int JT) { return 2 * JT + 8; }
__host__ __device__ constexpr int rec_words(int JT) { return 2 * JT + 8 + JT / 4; }
// Scalar slots
constexpr int kScC = 0, kScFv = 1, kScGv = 2, kScRt = 3, kScFt = 4, kScIvDtc = 5, kScUHdr = 6;
// Cell offset of a row without a feasible successor (or past the tile).
constexpr int kNoCell = -128;
// Record header (dword 8): the window row (0 .. 2H) of the first successor
// cell of a regular record, or one of these.
constexpr int kRecIrregular = -1;   // rows read one by one
constexpr int kRecEmpty = -2;       // no row of the tile has a successor

// Battery coordinates of one (speed node, SoC tile, sorted position), written
// as one packed record per (speed node, tile, position) so that the sweep
// stages a run of controls with one contiguous copy: per SoC node the lower
// cell (as an offset from the node) and the weights (fx, gx) times gt; the
// header says how the sweep reads the record.  One lane per (record, SoC row): the JT lanes of a
// record are consecutive and aligned (JT divides the wave), consecutive
// records are consecutive in memory, and the battery power and time step of
// the control come from the sort (no second powertrain evaluation).
__global__ void __launch_bounds__(256) k_stage_bat_sorted(StageBase B)
{
#pragma clang fp contract(off)
    const StageJob &jb = B.jobs[blockIdx.y];
    const DevInst &P = B.insts[jb.inst];
    const int JT = jb.jt, ntiles = jb.ntiles;
    const SortedEntry *__restrict__ st = (const SortedEntry *)(B.scr + jb.st);
    const double2 *__restrict__ pw = (const double2 *)(B.scr + jb.pw);
    const int *__restrict__ nfeas = (const int *)(B.scr + jb.nf);
    float *__restrict__ rec = (float *)(B.scr + jb.rec);
    const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long total = (long)P.n_v * ntiles * P.n_u * JT;
    if (idx >= total) return;          // whole records: total is a multiple of JT
    const int q = (int)(idx % JT);
    const long t2 = idx / JT;
    const int r = (int)(t2 % P.n_u);
    const long t3 = t2 / P.n_u;
    const int tile = (int)(t3 % ntiles);
    const int i = (int)(t3 / ntiles);
    if (r >= nfeas[i]) return;         // the same for the JT lanes of the record
    const long ir = (long)i * P.n_u + r;
    const int j0 = tile * JT;
    const int jc = min(JT, P.n_s - j0);
    int jx = -1;
    double fx = 0.0;
    const double2 pd = pw[ir];
    // the time weight gt of the control, exactly as the sort derived it
    double gt;
    {
        const double delta = pd.y / P.ht;
        gt = 1.0 - (delta - floor(delta));
    }
    if (q < jc) {
        const int j = j0 + q;
        double I;
        const double xi = P.s_lo + j * P.hs;
        if (battery_current(P, pd.x, xi, I)) {
            const double rs = (double)j - (pd.y * I) / (P.Cnom * P.hs);
            if (rs >= 0.0 && rs <= P.n_s - 1) cell_of(rs, P.n_s, jx, fx);
        }
        // the row's cell is stored as an int8 offset from the row (the host
        // bound on the shift keeps it within +-121); one outside that range
        // would wrap, so it raises the plan's device error instead
        if (jx >= 0 && (jx - j > 126 || jx - j < -127)) {
            atomicOr(B.err, kDevErrCellOffset);
            jx = -1;
        }
    }
    // The record is regular when its feasible rows have consecutive cells
    // jx = b + q with |b - j0| <= H and the tile holds at least half of JT
    // rows: the sweep then reads rows b .. b + JT from the staged window,
    // whose LDS row 0 is SoC row j0 - H (possibly below the grid), for all
    // JT rows.  Rows without a successor, and rows past a short last tile,
    // read whatever those LDS rows hold and carry not-a-number weights, so
    // their candidate never wins a comparison.  (A tile of fewer rows is
    // cheaper on the general path, which works row by row.)
    const int lane = threadIdx.x & 63;
    const int base = lane & ~(JT - 1);
    const unsigned long long grp = (JT == 64 ? ~0ull : ((1ull << JT) - 1ull)) << base;
    const unsigned long long feas = __ballot(jx >= 0) & grp;
    const int first = feas ? __ffsll((long long)feas) - 1 : base;
    const int b = __shfl(jx - q, first);
    const unsigned long long bad = __ballot(jx >= 0 && jx - q != b) & grp;
    int hdr = kRecIrregular;
    if (feas == 0) hdr = kRecEmpty;
    else if (bad == 0 && 2 * jc >= JT && b >= j0 - jb.H && b <= j0 + jb.H) hdr = b - (j0 - jb.H);
    const int CW = rec_words(JT);
    float *out = rec + (((long)i * ntiles + tile) * P.n_u + r) * CW;
    // SoC weights times the time weight gt (rounded once, from FP64), by
    // groups of R rows: lower-cell weights, then upper-cell weights
    const int R = JT > 8 ? 8 : JT;
    const int wg = (q / R) * 2 * R, wr = q % R;
    const float nan = __int_as_float(0x7fc00000);
    out[wg + wr] = jx >= 0 ? (float)((1.0 - fx) * gt) : nan;
    out[wg + R + wr] = jx >= 0 ? (float)(fx * gt) : nan;
    // the row's cell as a byte offset from the row (|offset| <= H + 1 < 127)
    reinterpret_cast<int8_t *>(out + rec_cells(JT))[q] = (int8_t)(jx >= 0 ? jx - (j0 + q) : kNoCell);
    const SortedEntry &e = st[ir];
    for (int w = q; w < 8; w += JT) {
        float x = 0.0f;
        switch (w) {
        case kScC: x = e.c; break;
        case kScFv: x = e.fv; break;
        case kScGv: x = e.gv; break;
        case kScRt: x = e.rt; break;
        case kScFt: x = e.ft; break;
        case kScIvDtc: x = __int_as_float((e.iv & 0xffff) | (e.dtc << 16)); break;
        case kScUHdr: x = __int_as_float((e.u & 0xffff) | (int)((unsigned)hdr << 16)); break;
        default: break;
        }
        out[rec_scalars(JT) + w] = x;
    }
}

// ------------------------------------------------------------------ sweep --

// Time lerp of R rows at once, in place: T[q] += rt * T[q] of the next lane
// (lane 63 adds 0), one v_fmac_f32_dpp per row (the compiler splits this into
// a DPP move and an FMA).  A DPP read of a VGPR needs two wait states after
// the VALU write of it: the leading s_nop covers the rows' last writes, and
// inside the block every instruction reads only its own row.  The whole wave
// must be active.
#define ECODP_TL(i) "v_fmac_f32_dpp %" #i ", %" #i ", %[rt] wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
template <int R> __device__ inline void time_lerp(float (&T)[R], float rt);
template <> __device__ inline void time_lerp<2>(float (&T)[2], float rt)
{
    asm("s_nop 1\n\t" ECODP_TL(0) ECODP_TL(1) : "+v"(T[0]), "+v"(T[1]) : [rt] "v"(rt));
}
template <> __device__ inline void time_lerp<5>(float (&T)[5], float rt)
{
    asm("s_nop 1\n\t" ECODP_TL(0) ECODP_TL(1) ECODP_TL(2) ECODP_TL(3) ECODP_TL(4)
        : "+v"(T[0]), "+v"(T[1]), "+v"(T[2]), "+v"(T[3]), "+v"(T[4]) : [rt] "v"(rt));
}
template <> __device__ inline void time_lerp<9>(float (&T)[9], float rt)
{
    asm("s_nop 1\n\t" ECODP_TL(0) ECODP_TL(1) ECODP_TL(2) ECODP_TL(3) ECODP_TL(4) ECODP_TL(5) ECODP_TL(6)
        ECODP_TL(7) ECODP_TL(8)
        : "+v"(T[0]), "+v"(T[1]), "+v"(T[2]), "+v"(T[3]), "+v"(T[4]), "+v"(T[5]), "+v"(T[6]), "+v"(T[7]),
          "+v"(T[8]) : [rt] "v"(rt));
}
template <> __device__ inline void time_lerp<17>(float (&T)[17], float rt)
{
    asm("s_nop 1\n\t" ECODP_TL(0) ECODP_TL(1) ECODP_TL(2) ECODP_TL(3) ECODP_TL(4) ECODP_TL(5) ECODP_TL(6)
        ECODP_TL(7) ECODP_TL(8) ECODP_TL(9) ECODP_TL(10) ECODP_TL(11) ECODP_TL(12) ECODP_TL(13) ECODP_TL(14)
        ECODP_TL(15) ECODP_TL(16)
        : "+v"(T[0]), "+v"(T[1]), "+v"(T[2]), "+v"(T[3]), "+v"(T[4]), "+v"(T[5]), "+v"(T[6]), "+v"(T[7]),
          "+v"(T[8]), "+v"(T[9]), "+v"(T[10]), "+v"(T[11]), "+v"(T[12]), "+v"(T[13]), "+v"(T[14]),
          "+v"(T[15]), "+v"(T[16]) : [rt] "v"(rt));
}
#undef ECODP_TL

// Lane q of every row of 16 lanes broadcast to the whole row (DPP
// row_newbcast): a record field that lane q holds becomes wave-uniform data
// in a VGPR without an LDS broadcast read.
template <int L> __device__ inline float row_bcast(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x150 + L, 0xf, 0xf, false));
}

// SoC lerp of R rows: Q[q] = W(lane q) T[q] + W(lane R + q) T[q + 1], the
// weights broadcast from the record VGPR W by DPP.  The products with the
// lower-cell weights are plain code (the compiler folds the broadcast into a
// v_mul_f32_dpp); the second terms are one v_fmac_f32_dpp per row here.  W is
// loaded from LDS, but a register copy of it made by the compiler just before
// this block would be a VALU write, hence the two wait states before the
// first DPP read.
template <int R, int Q0> struct SocLow {
    static __device__ inline void run(float (&Q)[R], float W, const float (&T)[R + 1])
    {
        Q[Q0] = row_bcast<Q0>(W) * T[Q0];
        SocLow<R, Q0 + 1>::run(Q, W, T);
    }
};
template <int R> struct SocLow<R, R> {
    static __device__ inline void run(float (&)[R], float, const float (&)[R + 1]) {}
};
#define ECODP_SF(q, l) "v_fmac_f32_dpp %" #q ", %[w], %" #l " row_newbcast:" #l " row_mask:0xf bank_mask:0xf\n\t"
template <int R> __device__ inline void soc_lerp(float (&Q)[R], float W, const float (&T)[R + 1]);
template <> __device__ inline void soc_lerp<4>(float (&Q)[4], float W, const float (&T)[5])
{
    SocLow<4, 0>::run(Q, W, T);
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %[w], %[t1] row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %[w], %[t2] row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %[w], %[t3] row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %[w], %[t4] row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(Q[0]), "+v"(Q[1]), "+v"(Q[2]), "+v"(Q[3])
        : [w] "v"(W), [t1] "v"(T[1]), [t2] "v"(T[2]), [t3] "v"(T[3]), [t4] "v"(T[4]));
}
template <> __device__ inline void soc_lerp<8>(float (&Q)[8], float W, const float (&T)[9])
{
    SocLow<8, 0>::run(Q, W, T);
    asm("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %[w], %[t1] row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %[w], %[t2] row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %[w], %[t3] row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %[w], %[t4] row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %[w], %[t5] row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %5, %[w], %[t6] row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %6, %[w], %[t7] row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %7, %[w], %[t8] row_newbcast:15 row_mask:0xf bank_mask:0xf\n\t"
        : "+v"(Q[0]), "+v"(Q[1]), "+v"(Q[2]), "+v"(Q[3]), "+v"(Q[4]), "+v"(Q[5]), "+v"(Q[6]), "+v"(Q[7])
        : [w] "v"(W), [t1] "v"(T[1]), [t2] "v"(T[2]), [t3] "v"(T[3]), [t4] "v"(T[4]), [t5] "v"(T[5]),
          [t6] "v"(T[6]), [t7] "v"(T[7]), [t8] "v"(T[8]));
}
#undef ECODP_SF

// Registers per thread that prefetch the next run of control records.
constexpr int kPrefetch = 4;
// Rows of a next-stage plane one thread loads per pass when staging.
constexpr int kStageRows = 8;
// Value of the staged columns past the last time node (half the largest
// float, so that sums of two of them stay finite).
constexpr float kPad = 1.7014118e38f;

// One item of the grouped sweep: speed node (by rank of work) x SoC tile x
// control slice `item` of stage job `jb` (instance parameters PI), on the
// workgroup's LDS `lds`; every thread of the workgroup calls it.
template <int JT, int PITCH>
__device__ __forceinline__ void sweep_item(const StageBase &B, const StageJob &jb, const DevInst &PI, int item,
                                           float *lds)
{
    constexpr int CW = rec_words(JT);
    SweepArgs P;
    P.n_v = PI.n_v;
    P.n_t = PI.n_t;
    P.n_s = PI.n_s;
    P.n_u = PI.n_u;
    P.zero_row = PI.zero_row;
    P.wait = PI.wait;
    P.Jinf = (float)PI.Jinf;
    P.v_lo = PI.v_lo;
    P.hv = PI.hv;
    P.vmax = PI.vmax;
    const int k = jb.k, H = jb.H, ntiles = jb.ntiles, rw = jb.rw, nsplit = jb.nsplit;
    const float *__restrict__ Jn = B.Jn ? B.Jn : (const float *)(B.J + jb.jn);
    float *__restrict__ Jk = B.Jk ? B.Jk : (float *)(B.J + jb.jk);
    int16_t *__restrict__ pik = B.pik ? B.pik : (int16_t *)(B.pi + jb.pik);
    const int *__restrict__ nfeas = (const int *)(B.scr + jb.nf);
    const float *__restrict__ rec = (const float *)(B.scr + jb.rec);
    const TLEntry *__restrict__ tl = jb.tl >= 0 ? B.tl + jb.tl : nullptr;
    float *__restrict__ part_v = (float *)(B.scr + jb.pv);
    int16_t *__restrict__ part_u = (int16_t *)(B.scr + jb.pu);
    const int nt = P.n_t, ns = P.n_s, nu = P.n_u;
    const int ir = item / (ntiles * nsplit);
    const int rem = item - ir * ntiles * nsplit;
    // speed nodes in decreasing order of work (written after the counts)
    const int i = __builtin_amdgcn_readfirstlane(nfeas[P.n_v + ir]);
    const int tile = rem / nsplit;
    const int split = rem - tile * nsplit;
    const int j0 = tile * JT;
    const int jc = min(JT, ns - j0);
    // SoC rows wlo..whi are staged; LDS row r of a plane holds SoC row
    // j0 - H + r (rows below 0 or above n_s - 1 are never staged)
    const int wlo = max(0, j0 - H);
    const int whi = min(ns - 1, j0 + jc + H);
    const int nrows = whi - wlo + 1;
    const int wbase = j0 - H;
    const int sh = wlo - wbase;
    // A tile of more than 8 rows runs on JT / 8 groups of waves, group g
    // taking rows 8 g ... 8 g + 7 of the tile: the groups share one staged
    // window (for a 16-row tile 2H + 1 fewer staged rows than two 8-row
    // workgroups) and each wave keeps the registers of an 8-row tile.  A wave covers 63
    // consecutive time nodes of its group's rows (its last lane is the halo
    // of the time lerp).
    constexpr int R = JT > 8 ? 8 : JT;          // tile rows per wave
    constexpr int NG = JT / R;                  // wave groups per workgroup
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int gthreads = (int)blockDim.x / NG;  // threads per group
    const int grp = __builtin_amdgcn_readfirstlane(NG > 1 ? (int)threadIdx.x / gthreads : 0);
    const int qb = grp * R;                     // first tile row of this wave
    const int m = (wave - grp * (gthreads >> 6)) * 63 + lane;
    const bool out_lane = lane < 63 && m < nt;
    const float Jinf = P.Jinf;
    // The running minimum of a row as one FP64 word: the high half holds the
    // FP32 value's bits with the sign cleared, the low half the control's
    // position in the node's visit order (plus one) above its index u.  Every
    // value is non-negative (stage and terminal costs are; a NaN candidate's
    // cleared bits sit above +inf), and the FP64 order of such words is the
    // order of the values, then of the positions: one v_min_f64 per row keeps
    // the first minimum in visit order (the order a strict < keeps) without a
    // compare and two selects, and J_inf at position 0 (no control) loses to
    // any value below J_inf and beats J_inf itself.
    double bk[R];
#pragma unroll
    for (int q = 0; q < R; q++) bk[q] = __hiloint2double(__float_as_int(Jinf), 0);
    double v;
    {
#pragma clang fp contract(off)
        v = P.v_lo + i * P.hv;
    }
    const bool row_ok = !(v > P.vmax[k]);
    const int nf = __builtin_amdgcn_readfirstlane(row_ok ? nfeas[i] : 0);
    const int r_begin = (int)(((long)nf * split) / nsplit);
    const int r_end = (int)(((long)nf * (split + 1)) / nsplit);
    const long SV = (long)ns * nt;
    const int slot_sz = rw * PITCH;              // floats per staged plane
    float *chunk = lds + 2 * slot_sz;             // kPrefetch * blockDim floats
    const int cc = __builtin_amdgcn_readfirstlane((kPrefetch * (int)blockDim.x) / CW);   // controls per staged run
    const float *recs = rec + ((long)i * ntiles + tile) * nu * CW;
    const int wofs = 2 * R * grp;               // this wave group's weights in a record
    const int wlane = lane & (2 * R - 1);
    const int slane = lane & 15;
    int nrec = 0;   // records of this item with at least one successor (evaluated)
    int plane[2] = {-1, -1};
    int cur_p = -2;
    int SA = 0, SB = 0;   // LDS float offsets of the staged planes cur_p, cur_p + 1

    float pre[kPrefetch];
    auto fetch = [&](int c0) {
        const int cnw = min(cc, r_end - c0) * CW;
        const float *src = recs + (long)c0 * CW;
#pragma unroll
        for (int q = 0; q < kPrefetch; q++) {
            const int x = threadIdx.x + q * blockDim.x;
            pre[q] = x < cnw ? src[x] : 0.0f;
        }
    };

    if (r_begin < r_end) fetch(r_begin);
    for (int c0 = r_begin; c0 < r_end; c0 += cc) {
        __syncthreads();                           // the previous run is no longer read
#pragma unroll
        for (int q = 0; q < kPrefetch; q++) chunk[threadIdx.x + q * blockDim.x] = pre[q];
        __syncthreads();
        if (c0 + cc < r_end) fetch(c0 + cc);        // in flight while this run is processed
        const int cn = __builtin_amdgcn_readfirstlane(min(cc, r_end - c0));
        // each control: one LDS load of the wave's 2R weights (lane l takes
        // weight l mod 2R) and one of the record's scalars and cells (lane l
        // takes word l mod 16 after the weights), issued one control ahead
        float W = 0.0f, S = 0.0f;
        if (cn > 0) {
            W = chunk[wofs + wlane];
            S = chunk[rec_scalars(JT) + slane];
        }
        for (int cr = 0; cr < cn; cr++) {
            const int ivdtc = __builtin_amdgcn_readlane(__float_as_int(S), kScIvDtc);
            const int uhdr = __builtin_amdgcn_readlane(__float_as_int(S), kScUHdr);
            const float *nx = chunk + min(cr + 1, cn - 1) * CW;
            const int hdr = uhdr >> 16;
            if (hdr == kRecEmpty) {                  // no row of this tile has a successor
                W = nx[wofs + wlane];
                S = nx[rec_scalars(JT) + slane];
                continue;
            }
            nrec++;
            const int p = ivdtc & 0xffff;
            const int dtc = ivdtc >> 16;
            const int u = uhdr & 0xffff;
            if (p != cur_p) {
                // stage planes p and p+1 (SoC rows wlo..whi, every time node),
                // keeping a plane already resident from the previous group
                int sp = plane[0] == p ? 0 : (plane[1] == p ? 1 : -1);
                int sq = plane[0] == p + 1 ? 0 : (plane[1] == p + 1 ? 1 : -1);
                const bool need_p = sp < 0, need_q = sq < 0;
                if (need_p && need_q) {
                    sp = 0;
                    sq = 1;
                } else if (need_p) {
                    sp = 1 - sq;
                } else if (need_q) {
                    sq = 1 - sp;
                }
                __syncthreads();
                // thread t of a group copies time node t (a group has at
                // least n_t threads) of kStageRows rows per pass, all loads in
                // flight before the LDS stores; group g takes passes g, g +
                // NG, ...
                int t = threadIdx.x;
                if (NG > 1) {
                    // the thread's index within its group, formed here (not
                    // kept in a register across the control loop)
                    asm volatile("v_subrev_u32 %0, %1, %0" : "+v"(t) : "s"(grp * gthreads));
                }
                if (grp == 0 && t >= nt && t < PITCH) {
                    // columns past the last time node hold a huge finite value:
                    // a candidate whose successor time leaves the grid (or sits
                    // on the last node with a positive fraction) is then far
                    // above J_inf, infinite, or not a number (a zero SoC
                    // weight times an infinite time lerp), none of which wins,
                    // while 0 x huge stays exact for a zero fraction on the
                    // last node
                    for (int rr = 0; rr < nrows; rr++) {
                        if (need_p) lds[sp * slot_sz + (rr + sh) * PITCH + t] = kPad;
                        if (need_q) lds[sq * slot_sz + (rr + sh) * PITCH + t] = kPad;
                    }
                }
                if (t < nt) {
                    const float *srcp = Jn + (long)p * SV + (long)wlo * nt + t;
                    const float *srcq = srcp + SV;
                    if (need_p || need_q)
                        for (int r0 = grp * kStageRows; r0 < nrows; r0 += NG * kStageRows) {
                            float va[kStageRows], vb[kStageRows];
#pragma unroll
                            for (int q = 0; q < kStageRows; q++) {
                                const long off = (long)min(r0 + q, nrows - 1) * nt;
                                va[q] = need_p ? srcp[off] : 0.0f;
                                vb[q] = need_q ? srcq[off] : 0.0f;
                            }
#pragma unroll
                            for (int q = 0; q < kStageRows; q++) {
                                if (r0 + q < nrows) {
                                    if (need_p) lds[sp * slot_sz + (r0 + q + sh) * PITCH + t] = va[q];
                                    if (need_q) lds[sq * slot_sz + (r0 + q + sh) * PITCH + t] = vb[q];
                                }
                            }
                        }
                }
                plane[sp] = p;
                plane[sq] = p + 1;
                SA = sp * slot_sz;
                SB = sq * slot_sz;
                cur_p = p;
                __syncthreads();
            }
            // wave-uniform scalars of the control as VGPRs (DPP broadcasts)
            const float c0f = row_bcast<kScC>(S), fv = row_bcast<kScFv>(S), gv = row_bcast<kScGv>(S);
            const float rt = row_bcast<kScRt>(S);
            const int pos = m + dtc;
            float Qv[R];
            // a wave group of a 16-row tile with at most half of its rows
            // inside the tile (the last tile of the grid) takes the general
            // path, which runs only those rows
            if (hdr >= 0 && (NG == 1 || 2 * (jc - qb) > R)) {
                // successor times past the grid read the padding columns
                const int posc = min(pos, PITCH - 1);
                const int a0 = SA + (hdr + qb) * PITCH + posc;
                const int b0 = SB + (hdr + qb) * PITCH + posc;
                // speed lerp on the R+1 SoC rows with the stage cost added
                // (the time and SoC weights of a node sum to one, so c passes
                // through both lerps), then the time lerp with the
                // neighbouring lane (scaled by 1/gt), then the SoC lerp per
                // node (weights scaled by gt)
                float T[R + 1];
#pragma unroll
                for (int q = 0; q <= R; q++) T[q] = fmaf(fv, lds[b0 + q * PITCH], fmaf(gv, lds[a0 + q * PITCH], c0f));
                time_lerp(T, rt);
                soc_lerp<R>(Qv, W, T);
            } else {
                const float ft = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(S), kScFt));
                const bool okt = out_lane && (pos < nt - 1 || (pos == nt - 1 && ft == 0.0f));
                const int posc = min(pos, nt - 1);
                // the rows' cells, four int8 offsets per dword, held by the
                // scalar VGPR's lanes 8 ...
                int cw[R / 4];
#pragma unroll
                for (int w = 0; w < R / 4; w++)
                    cw[w] = __builtin_amdgcn_readlane(__float_as_int(S), 8 + qb / 4 + w);
#pragma unroll
                for (int q = 0; q < R; q++) {
                    const int off = (int)(int8_t)(cw[q / 4] >> (8 * (q % 4)));
                    const int jx = qb + q < jc && off != kNoCell ? j0 + qb + q + off : -1;
                    Qv[q] = Jinf;
                    if (jx >= 0) {
                        float T2[2];
                        if (jx >= wlo && jx + 1 <= whi) {
                            const int a = SA + (jx - wbase) * PITCH + posc;
                            const int b = SB + (jx - wbase) * PITCH + posc;
                            T2[0] = fmaf(fv, lds[b], fmaf(gv, lds[a], c0f));
                            T2[1] = fmaf(fv, lds[b + PITCH], fmaf(gv, lds[a + PITCH], c0f));
                        } else {
                            const float *a = Jn + (long)p * SV + (long)jx * nt + posc;
                            T2[0] = fmaf(fv, a[SV], fmaf(gv, a[0], c0f));
                            T2[1] = fmaf(fv, a[SV + nt], fmaf(gv, a[nt], c0f));
                        }
                        // (every lane's value stays finite through the time
                        // lerp, which reads the neighbouring lane's)
                        time_lerp(T2, rt);
                        const float w0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(W), q));
                        const float w1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(W), R + q));
                        const float qv = fmaf(w1, T2[1], w0 * T2[0]);
                        // a lane whose successor time is off the grid never wins
                        Qv[q] = okt ? qv : __builtin_inff();
                    }
                }
            }
            // the next control's record
            W = nx[wofs + wlane];
            S = nx[rec_scalars(JT) + slane];
            {
                const int rk = ((c0 + cr + 1) << 16) | u;   // positions and u below 2^15
#pragma unroll
                for (int q = 0; q < R; q++) {
                    const double cand = __hiloint2double(__float_as_int(Qv[q]) & 0x7fffffff, rk);
                    asm("v_min_f64 %0, %1, %2" : "=v"(bk[q]) : "v"(cand), "v"(bk[q]));
                }
            }
        }
    }
    if (threadIdx.x == 0 && nrec > 0)
        atomicAdd(B.count + jb.inst, (unsigned long long)nrec * (unsigned long long)(jc * nt));
    // the minimum's value and control (position 0: none)
    float best[R];
    int bu[R];
#pragma unroll
    for (int q = 0; q < R; q++) {
        best[q] = __int_as_float(__double2hiint(bk[q]));
        const int rk = __double2loint(bk[q]);
        bu[q] = rk > 0 ? (rk & 0xffff) : -1;
    }
    if (out_lane && nsplit > 1) {
        // partial minimum of this control slice; the combine kernel finishes
        const long plane_nodes = (long)P.n_v * SV;
#pragma unroll
        for (int q = 0; q < R; q++) {
            if (qb + q < jc) {
                const long n = ((long)i * ns + j0 + qb + q) * nt + m;
                part_v[split * plane_nodes + n] = best[q];
                part_u[split * plane_nodes + n] = (int16_t)bu[q];
            }
        }
    } else if (out_lane) {
        TLEntry t;
        const bool has_tl = tl != nullptr;
        if (has_tl) t = tl[m];
        const bool stop = has_tl && tl_stop(t, v, PI.amin);
#pragma unroll
        for (int q = 0; q < R; q++) {
            if (qb + q < jc) {
                const int j = j0 + qb + q;
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
    }
}

// The job and parameter tables come in as separate read-only arguments so
// that their fields are loaded through the scalar unit.
// 16-row tiles run three 8-wave workgroups per CU when a lane holds at most
// 80 registers (six waves per SIMD): the compiler is held to that.
template <int JT, int PITCH>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(JT == 16 ? 6 : 1, 8)))
k_sweep_lds(StageBase B, const StageJob *__restrict__ jobs, const DevInst *__restrict__ insts, int njobs,
            const int *__restrict__ item_begin, int total, int *__restrict__ queue)
{
    extern __shared__ float lds_base[];
    // A launch covers the items of njobs jobs; item_begin[q] is the first
    // item of job q (njobs + 1 entries, kept in LDS ahead of the planes).
    int *s_ib = reinterpret_cast<int *>(lds_base);
    const int ibw = item_begin ? ((njobs + 64) / 64) * 64 : 0;
    if (item_begin)
        for (int q = threadIdx.x; q <= njobs; q += blockDim.x) s_ib[q] = item_begin[q];
    float *lds = lds_base + ibw;
    // Persistent workgroups take (job, speed node, SoC tile, control slice)
    // items from eight queues, one contiguous band of items per XCD (blocks
    // are dealt round-robin over the 8 XCDs, so a band's next-stage planes
    // stay in one L2); a job's speed nodes come in decreasing order of work,
    // which keeps a band's nodes close in speed and leaves the shortest items
    // for the end.  A workgroup whose band is drained takes items from the
    // other bands; every workgroup exits once all queues are drained.  A
    // launch with no more items than workgroups skips the queues.
    __shared__ int s_item, s_job;
    const int home = blockIdx.x & 7;
    int qi = 0;
    __syncthreads();
    for (;;) {
    if (threadIdx.x == 0) {
        int item = -1, job = 0;
        if (total <= (int)gridDim.x) {
            // no more items than workgroups: workgroup b takes item b and
            // leaves (a drained queue polled by every workgroup would cost
            // more than the work)
            if (qi == 0 && (int)blockIdx.x < total) item = blockIdx.x;
            qi = 8;
        }
        while (qi < 8) {
            const int x = (home + qi) & 7;
            const int lo = (int)(((long)total * x) >> 3), hi = (int)(((long)total * (x + 1)) >> 3);
            const int got = lo + atomicAdd(&queue[x], 1);
            if (got < hi) {
                item = got;
                break;
            }
            qi++;
        }
        if (item >= 0 && item_begin) {
            // the last job whose first item is <= item
            int a = 0, b = njobs - 1;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (s_ib[mid] <= item) a = mid;
                else b = mid - 1;
            }
            job = a;
            item -= s_ib[a];
        }
        s_item = item;
        s_job = job;
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    const int jbi = __builtin_amdgcn_readfirstlane(s_job);
    __syncthreads();
    if (item < 0) break;
    sweep_item<JT, PITCH>(B, jobs[jbi], insts[jobs[jbi].inst], item, lds);
    }   // item loop
}

// Persistent grouped sweep over every stage of many instances (the batched
// solve in one launch per kernel class).  Each XCD has its own queue of
// (instance, stage) jobs and the instances of a queue are served by the
// workgroups running on that XCD only, which read the hardware XCC id: the
// values a stage writes are then read by the next stage through the same
// L2, so a workgroup publishes an item by waiting for its stores (vmcnt)
// before it counts the item, and a workgroup that takes an item of stage k
// waits (bounded) until the instance's items of stages N-1..k+1 are all
// counted, then invalidates its CU's L1 before it reads J_{k+1}.  Within a
// queue the jobs come round by round (stage N_b - 1 - r of every instance of
// the queue in round r), so the items a wait depends on were all taken
// earlier by running workgroups.  A wait that exceeds the spin limit, or an
// error raised by another workgroup, makes every workgroup leave; the error
// word then holds kDevErrWait.  4- and 16-row tiles are held to 80 registers
// a lane (six waves per SIMD), as in the round-by-round sweep.
template <int JT, int PITCH>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(JT == 8 ? 1 : 6, 8)))
k_sweep_persist(StageBase B, const DevInst *__restrict__ insts, PersistQueues Q)
{
    extern __shared__ float lds[];
    __shared__ int s_item, s_job;
    int xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    const int x = (xcc & 0xf) % Q.n_xcd;
    const int jb0 = Q.xjb[x], jb1 = Q.xjb[x + 1];
    const int total = Q.xtot[x];
    int jcur = jb0;       // thread 0: job of its last claim (claims only grow)
    for (;;) {
        if (threadIdx.x == 0) {
            int item = -1, job = -1;
            if (jb0 < jb1 && __hip_atomic_load(Q.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                const int g = atomicAdd(Q.claim + x, 1);
                if (g < total) {
                    while (jcur + 1 < jb1 && Q.jobs[jcur + 1].item0 <= g) jcur++;
                    const PJob &pj = Q.jobs[jcur];
                    const int need = pj.need;
                    int *done = Q.done + pj.j.inst;
                    // the test hook: the queue's first job also waits for a
                    // count nothing ever reaches
                    const bool stall = Q.stall && jcur == jb0;
                    long long spins = 0;
                    bool ok = true;
                    while (stall || __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if (++spins > Q.spin_limit ||
                            __hip_atomic_load(Q.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            atomicOr(Q.err, kDevErrWait);
                            ok = false;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                    if (ok) {
                        job = jcur;
                        item = g - pj.item0;
                    }
                }
            }
            s_item = item;
            s_job = job;
        }
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        const int job = __builtin_amdgcn_readfirstlane(s_job);
        __syncthreads();
        if (item < 0) break;
        // every wave drops its CU's L1 copies before it reads, so that J_{k+1}
        // comes from the XCD's L2, which holds the other workgroups' stores.
        // The invalidate must be of device scope: the workgroup-scope form
        // leaves the L1 of a workgroup that runs on one CU untouched (measured:
        // with it the last stages of an instance read stale J_{k+1} lines)
        asm volatile("buffer_inv sc1" ::: "memory");
        const PJob &pj = Q.jobs[job];
        sweep_item<JT, PITCH>(B, pj.j, insts[pj.j.inst], item, lds);
        // every store of the item has reached the L2 before the item counts
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(Q.done + pj.j.inst, 1);
    }
}

// Minimum over the control splits (the first split wins a tie, so the result
// does not depend on the number of splits), then the signal override and the
// store of J_k and pi_k.
__global__ void k_sweep_combine(StageBase B)
{
    const StageJob &jb = B.jobs[blockIdx.y];
    const int nsplit = jb.nsplit;
    if (nsplit <= 1) return;
    const DevInst &P = B.insts[jb.inst];
    const float *__restrict__ Jn = B.Jn ? B.Jn : (const float *)(B.J + jb.jn);
    float *__restrict__ Jk = B.Jk ? B.Jk : (float *)(B.J + jb.jk);
    int16_t *__restrict__ pik = B.pik ? B.pik : (int16_t *)(B.pi + jb.pik);
    const TLEntry *__restrict__ tl = jb.tl >= 0 ? B.tl + jb.tl : nullptr;
    const float *__restrict__ part_v = (const float *)(B.scr + jb.pv);
    const int16_t *__restrict__ part_u = (const int16_t *)(B.scr + jb.pu);
    const float Jinf = (float)P.Jinf;
    const long S = (long)P.n_v * P.n_s * P.n_t;
    for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < S; n += (long)gridDim.x * blockDim.x) {
        float J = part_v[n];
        int pu = part_u[n];
        for (int sp = 1; sp < nsplit; sp++) {
            const float x = part_v[sp * S + n];
            if (x < J) {
                J = x;
                pu = part_u[sp * S + n];
            }
        }
        if (tl != nullptr) {
            const int m = (int)(n % P.n_t);
            const TLEntry t = tl[m];
            const long ij = n / P.n_t;
            const int i = (int)(ij / P.n_s);
            double v;
            {
#pragma clang fp contract(off)
                v = P.v_lo + i * P.hv;
            }
            if (tl_stop(t, v, P.amin)) {
                J = Jinf;
                pu = -1;
                if (i == P.zero_row && P.wait && t.wc >= 0) {
                    const float *pw = Jn + ij * P.n_t + t.wc;
                    const float w = wait_value(t, pw);
                    if (w < Jinf) {
                        J = w;
                        pu = -2;
                    }
                }
            }
        }
        Jk[n] = J;
        pik[n] = (int16_t)pu;
    }
}

// ----------------------------------------------------------------- launch --

int launch_stage_jobs(const StageBase &B, int njobs, int max_nv, long max_records, hipStream_t s)
{
    hipLaunchKernelGGL(k_stage_sort, dim3(max_nv, njobs), dim3(1024), 0, s, B);
    if (hipGetLastError() != hipSuccess) return -1;
    hipLaunchKernelGGL(k_stage_rank, dim3(njobs), dim3(256), 0, s, B);
    if (hipGetLastError() != hipSuccess) return -1;
    hipLaunchKernelGGL(k_stage_bat_sorted, dim3((unsigned)((max_records + 255) / 256), njobs), dim3(256), 0, s, B);
    // (max_records counts record lanes: records x SoC rows per record)
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

size_t lds_sweep_bytes_p(int JT, int H, int pitch, int threads)
{
    return sizeof(float) * (2 * (size_t)sweep_rows(JT, H) * pitch + (size_t)kPrefetch * threads + 16);
}

size_t lds_sweep_bytes(int JT, int H, int n_t)
{
    // the record chunk is followed by 16 spare floats: a record's scalar
    // load reads 16 words after its weights, past the last record's end
    return sizeof(float) * (2 * (size_t)sweep_rows(JT, H) * sweep_pitch(n_t) +
                            (size_t)kPrefetch * sweep_threads(JT, n_t) + 16);
}

size_t lds_job_index_bytes(int njobs) { return njobs > 1 ? sizeof(int) * (size_t)(((njobs + 64) / 64) * 64) : 0; }

template <int JT>
static int launch_sweep_p(int pitch, dim3 grid, dim3 block, size_t lds, hipStream_t s, const StageBase &B,
                          int njobs, const int *item_begin, int total, int *queue)
{
    switch (pitch) {
#define ECODP_PITCH(X)                                                                                        \
    case X:                                                                                                   \
        hipLaunchKernelGGL((k_sweep_lds<JT, X>), grid, block, lds, s, B, B.jobs, B.insts, njobs, item_begin, total, \
                           queue);                                                                              \
        return hipGetLastError() == hipSuccess ? 0 : -1;
        ECODP_PITCH(32)
        ECODP_PITCH(64)
        ECODP_PITCH(96)
        ECODP_PITCH(128)
        ECODP_PITCH(160)
        ECODP_PITCH(192)
        ECODP_PITCH(224)
        ECODP_PITCH(256)
        ECODP_PITCH(288)
        ECODP_PITCH(320)
        ECODP_PITCH(352)
        ECODP_PITCH(384)
        ECODP_PITCH(416)
        ECODP_PITCH(448)
        ECODP_PITCH(480)
        ECODP_PITCH(512)
        ECODP_PITCH(544)
        ECODP_PITCH(576)
        ECODP_PITCH(608)
        ECODP_PITCH(640)
        ECODP_PITCH(672)
        ECODP_PITCH(704)
        ECODP_PITCH(736)
        ECODP_PITCH(768)
        ECODP_PITCH(800)
        ECODP_PITCH(832)
        ECODP_PITCH(864)
        ECODP_PITCH(896)
        ECODP_PITCH(928)
        ECODP_PITCH(960)
        ECODP_PITCH(992)
        ECODP_PITCH(1024)
#undef ECODP_PITCH
    default: return -2;
    }
}

// Vector registers per lane of the grouped-sweep kernel instance (queried
// from the loaded code object; a conservative estimate if the query fails).
template <int JT>
static int sweep_vgprs_p(int pitch)
{
    hipFuncAttributes a;
    hipError_t e = hipErrorInvalidValue;
    switch (pitch) {
#define ECODP_PITCH(X)                                                                  \
    case X:                                                                             \
        e = hipFuncGetAttributes(&a, reinterpret_cast<const void *>(&k_sweep_lds<JT, X>)); \
        break;
        ECODP_PITCH(32)
        ECODP_PITCH(64)
        ECODP_PITCH(96)
        ECODP_PITCH(128)
        ECODP_PITCH(160)
        ECODP_PITCH(192)
        ECODP_PITCH(224)
        ECODP_PITCH(256)
        ECODP_PITCH(288)
        ECODP_PITCH(320)
        ECODP_PITCH(352)
        ECODP_PITCH(384)
        ECODP_PITCH(416)
        ECODP_PITCH(448)
        ECODP_PITCH(480)
        ECODP_PITCH(512)
        ECODP_PITCH(544)
        ECODP_PITCH(576)
        ECODP_PITCH(608)
        ECODP_PITCH(640)
        ECODP_PITCH(672)
        ECODP_PITCH(704)
        ECODP_PITCH(736)
        ECODP_PITCH(768)
        ECODP_PITCH(800)
        ECODP_PITCH(832)
        ECODP_PITCH(864)
        ECODP_PITCH(896)
        ECODP_PITCH(928)
        ECODP_PITCH(960)
        ECODP_PITCH(992)
        ECODP_PITCH(1024)
#undef ECODP_PITCH
    default: break;
    }
    if (e == hipSuccess && a.numRegs > 0) return a.numRegs;
    (void)hipGetLastError();
    return JT == 16 ? 128 : (JT == 8 ? 96 : 80);
}

template <int JT>
static int launch_persist_p(int pitch, dim3 grid, dim3 block, size_t lds, hipStream_t s, const StageBase &B,
                            const DevInst *insts, const PersistQueues &Q)
{
    switch (pitch) {
#define ECODP_PITCH(X)                                                                            \
    case X:                                                                                       \
        hipLaunchKernelGGL((k_sweep_persist<JT, X>), grid, block, lds, s, B, insts, Q);          \
        return hipGetLastError() == hipSuccess ? 0 : -1;
        ECODP_PITCH(32)
        ECODP_PITCH(64)
        ECODP_PITCH(96)
        ECODP_PITCH(128)
        ECODP_PITCH(160)
        ECODP_PITCH(192)
        ECODP_PITCH(224)
        ECODP_PITCH(256)
        ECODP_PITCH(288)
        ECODP_PITCH(320)
        ECODP_PITCH(352)
        ECODP_PITCH(384)
        ECODP_PITCH(416)
        ECODP_PITCH(448)
        ECODP_PITCH(480)
        ECODP_PITCH(512)
#undef ECODP_PITCH
    default: return -2;
    }
}

template <int JT>
static int persist_blocks_p(int pitch, int threads, size_t lds)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (pitch) {
#define ECODP_PITCH(X)                                                                                       \
    case X:                                                                                                  \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_sweep_persist<JT, X>), \
                                                         threads, lds);                                      \
        break;
        ECODP_PITCH(32)
        ECODP_PITCH(64)
        ECODP_PITCH(96)
        ECODP_PITCH(128)
        ECODP_PITCH(160)
        ECODP_PITCH(192)
        ECODP_PITCH(224)
        ECODP_PITCH(256)
        ECODP_PITCH(288)
        ECODP_PITCH(320)
        ECODP_PITCH(352)
        ECODP_PITCH(384)
        ECODP_PITCH(416)
        ECODP_PITCH(448)
        ECODP_PITCH(480)
        ECODP_PITCH(512)
#undef ECODP_PITCH
    default: break;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

int persist_blocks_per_cu(int JT, int pitch, int threads, size_t lds)
{
    if (JT == 8) return persist_blocks_p<8>(pitch, threads, lds);
    if (JT == 4) return persist_blocks_p<4>(pitch, threads, lds);
    if (JT == 16) return persist_blocks_p<16>(pitch, threads, lds);
    return 0;
}

int launch_sweep_persist(int JT, int pitch, int threads, const StageBase &B, const DevInst *insts,
                         const PersistQueues &Q, int grid, size_t lds, hipStream_t s)
{
    const dim3 g(grid), blk(threads);
    if (JT == 8) return launch_persist_p<8>(pitch, g, blk, lds, s, B, insts, Q);
    if (JT == 4) return launch_persist_p<4>(pitch, g, blk, lds, s, B, insts, Q);
    if (JT == 16) return launch_persist_p<16>(pitch, g, blk, lds, s, B, insts, Q);
    return -2;
}

int sweep_vgprs(int JT, int pitch)
{
    if (JT == 16) return sweep_vgprs_p<16>(pitch);
    if (JT == 8) return sweep_vgprs_p<8>(pitch);
    return sweep_vgprs_p<4>(pitch);
}

int launch_sweep_jobs(int JT, int pitch, int threads, const StageBase &B, int njobs, const int *item_begin,
                      int total, int *queue, int grid, size_t lds, hipStream_t s)
{
    const dim3 g(grid < total ? grid : total), blk(threads);
    if (njobs > 1 && !item_begin) return -2;
    const int *ib = njobs > 1 ? item_begin : nullptr;
    if (JT == 16) return launch_sweep_p<16>(pitch, g, blk, lds, s, B, njobs, ib, total, queue);
    if (JT == 8) return launch_sweep_p<8>(pitch, g, blk, lds, s, B, njobs, ib, total, queue);
    if (JT == 4) return launch_sweep_p<4>(pitch, g, blk, lds, s, B, njobs, ib, total, queue);
    return -2;
}

int launch_combine_jobs(const StageBase &B, int njobs, long max_nodes, hipStream_t s)
{
    long blocks = (max_nodes + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_sweep_combine, dim3((unsigned)blocks, njobs), dim3(256), 0, s, B);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

__global__ void k_fill_i32(int *p, long n, int v)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) p[q] = v;
}

int launch_fill_i32(int *p, long n, int v, hipStream_t s)
{
    long b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)b), dim3(256), 0, s, p, n, v);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ecodp
