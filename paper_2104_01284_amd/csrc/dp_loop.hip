// The closed-loop receding-horizon controller (Sec. V; the terminal cost from
// an offline DP over the whole route, Sec. III after Eq. 9) as a library
// object: the route's full-horizon solve, one plan per horizon length kept for
// the whole drive and moved along the route in place, and per step the
// stop-line wait (Eq. 5c, Eq. 8), the horizon's terminal table, the solve, the
// FP64 rollout whose first step is the plant step, and the violation checks.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ecodp.h"
#include "dp_internal.h"

using namespace ecodp;

namespace {

// One kept horizon plan and its buffers.
struct Window {
    dp_plan *p = nullptr;
    int N = 0;
    void *J = nullptr, *pi = nullptr, *scr = nullptr;
    float *V0 = nullptr;
    int16_t *u0 = nullptr;
    double *traj = nullptr;
    int32_t *status = nullptr;
    float *term = nullptr;     // the plan's own terminal table
    int64_t evals = 0;
};

int dev_alloc(void **ptr, size_t bytes)
{
    if (hipMalloc(ptr, std::max<size_t>(bytes, 256)) != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return api_fail(DP_ENOMEM, "loop: hipMalloc of %zu bytes failed", bytes);
    }
    return DP_OK;
}

// Seconds until green for a vehicle at speed v that has to stop at a signal
// at clock t, 0 when it may cross (Eq. 8: red iff (t - O) mod C in [0, R);
// in the Y seconds of yellow before red it has to stop once more time has
// passed since yellow began than v / (2 b), b = -a_min, Sec. III).
double stop_time(double C, double R, double O, double Y, double amin, double v, double t)
{
    double ph = std::fmod(t - O, C);
    if (ph < 0.0) ph += C;
    if (ph < R) return R - ph;
    if (Y > 0.0 && ph >= C - Y && ph - (C - Y) > v / (2.0 * -amin)) return (C - ph) + R;
    return 0.0;
}

}  // namespace

struct dp_loop {
    int device = 0;
    hipStream_t stream = nullptr;
    dp_problem_desc route;
    std::vector<double> grade, vmax, cyc, red, off, yel;
    std::vector<int32_t> lstage;
    std::vector<int> light_at;          // [N_route + 1]: signal index at a route stage, or -1
    int horizon = 0;
    double t_f = 0.0;
    int n_t = 0;
    bool timing = false;
    dp_plan *full = nullptr;            // the offline full-route solve
    void *fJ = nullptr, *fpi = nullptr, *fscr = nullptr;
    float *fV0 = nullptr;
    int16_t *fu0 = nullptr;
    size_t fslab = 0;                   // elements of one route value slab
    std::vector<Window> win;            // win[N - 1]: the plan of an N-step horizon
    double *host = nullptr;             // pinned: rollout rows 0 and 1, then V_0
    std::vector<double> wc, wr, wo, wy; // a window's per-stage signals
    dp_loop_totals tot;
    bool stopped = false;
};

static void loop_free(dp_loop *L)
{
    if (!L) return;
    (void)hipSetDevice(L->device);
    if (L->stream) (void)hipStreamSynchronize(L->stream);
    for (Window &w : L->win) {
        if (w.p) dp_destroy(w.p);
        for (void *q : {w.J, w.pi, w.scr, (void *)w.V0, (void *)w.u0, (void *)w.traj, (void *)w.status})
            if (q) (void)hipFree(q);
    }
    if (L->full) dp_destroy(L->full);
    for (void *q : {L->fJ, L->fpi, L->fscr, (void *)L->fV0, (void *)L->fu0})
        if (q) (void)hipFree(q);
    if (L->host) (void)hipHostFree(L->host);
    if (L->stream) (void)hipStreamDestroy(L->stream);
    delete L;
}

int dp_loop_create(const dp_problem_desc *route, int32_t horizon, double t_f, int32_t n_t, const dp_options *opt,
                   int32_t device, dp_loop **out)
{
    if (!out) return api_fail(DP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!route || !route->grade) return api_fail(DP_EINVAL, "loop: route or its grade is NULL");
    if (horizon < 1 || n_t < 2 || !(std::isfinite(t_f) && t_f > 0.0))
        return api_fail(DP_EINVAL, "loop: horizon %d, time grid [0, %g] x %d", horizon, t_f, n_t);
    if (opt && (opt->flags & ~(uint32_t)DP_TIMING)) return api_fail(DP_EINVAL, "loop: only DP_TIMING is an option flag");
    if (opt && opt->inst_opt) return api_fail(DP_EINVAL, "loop: per-instance options do not apply");
    const int NR = route->n_stages;
    if (NR < 1) return api_fail(DP_EINVAL, "loop: route of %d stages", NR);
    dp_loop *L = new (std::nothrow) dp_loop;
    if (!L) return api_fail(DP_ENOMEM, "host allocation");
    std::memset(&L->tot, 0, sizeof L->tot);
    L->device = device;
    L->horizon = horizon;
    L->t_f = t_f;
    L->n_t = n_t;
    L->timing = opt && (opt->flags & DP_TIMING);
    // the route, copied (a signal is looked up by stage below)
    L->route = *route;
    L->grade.assign(route->grade, route->grade + NR);
    L->vmax.resize(NR + 1);
    for (int k = 0; k <= NR; k++) L->vmax[k] = route->v_max ? route->v_max[k] : route->v_hi;
    L->light_at.assign(NR + 1, -1);
    for (int q = 0; q < route->n_lights; q++) {
        if (!route->light_stage || !route->light_cycle || !route->light_red || !route->light_offset) {
            loop_free(L);
            return api_fail(DP_EINVAL, "loop: signal arrays are NULL");
        }
        const int st = route->light_stage[q];
        if (st < 1 || st > NR - 1 || L->light_at[st] >= 0) {
            loop_free(L);
            return api_fail(DP_EINVAL, "loop: signal %d at stage %d", q, st);
        }
        L->light_at[st] = q;
        L->lstage.push_back(st);
        L->cyc.push_back(route->light_cycle[q]);
        L->red.push_back(route->light_red[q]);
        L->off.push_back(route->light_offset[q]);
        L->yel.push_back(route->light_yellow ? route->light_yellow[q] : 0.0);
    }
    L->route.grade = L->grade.data();
    L->route.v_max = L->vmax.data();
    L->route.light_stage = L->lstage.data();
    L->route.light_cycle = L->cyc.data();
    L->route.light_red = L->red.data();
    L->route.light_offset = L->off.data();
    L->route.light_yellow = L->yel.data();
    L->route.terminal_V = nullptr;
    L->route.flags &= ~(uint32_t)DP_TERMINAL_DEVICE;
    if (route->terminal_V) {
        loop_free(L);
        return api_fail(DP_EUNSUPPORTED, "loop: a route terminal table is not supported");
    }
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc((void **)&L->host, sizeof(double) * 32, hipHostMallocDefault);
    if (e != hipSuccess) {
        loop_free(L);
        return api_fail(DP_EDEVICE, "loop: stream or pinned buffer: %s", hipGetErrorString(e));
    }
    // the offline full-route solve
    const auto t0 = std::chrono::steady_clock::now();
    dp_options fo;
    std::memset(&fo, 0, sizeof fo);
    fo.flags = DP_STORE_ALL_V;
    int rc = dp_build_problem(&L->route, 1, &fo, device, &L->full);
    size_t bJ = 0, bpi = 0, bs = 0;
    if (!rc) rc = dp_workspace_size(L->full, &bJ, &bpi, &bs);
    if (!rc) rc = dev_alloc(&L->fJ, bJ);
    if (!rc) rc = dev_alloc(&L->fpi, bpi);
    if (!rc) rc = dev_alloc(&L->fscr, bs);
    if (!rc) rc = dev_alloc((void **)&L->fV0, sizeof(float));
    if (!rc) rc = dev_alloc((void **)&L->fu0, sizeof(int16_t));
    if (!rc) rc = dp_solve(L->full, L->fJ, L->fpi, L->fscr, L->fV0, L->fu0, L->stream);
    if (!rc && (e = hipStreamSynchronize(L->stream)) != hipSuccess)
        rc = api_fail(DP_EDEVICE, "loop: full-route solve: %s", hipGetErrorString(e));
    if (!rc) rc = dp_device_check(L->full, L->stream);   // a condition the kernels met (DP_EDEVICE)
    if (rc) {
        loop_free(L);
        return rc;
    }
    L->tot.offline_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    dp_instance_info fi;
    if ((rc = dp_instance_info_get(L->full, 0, &fi))) {
        loop_free(L);
        return rc;
    }
    L->fslab = fi.slab_elems;
    // one plan per horizon length: the route's grids and constants on the
    // horizon time grid, w_soc = 0 (the terminal cost comes from the offline
    // values), a placeholder signal at every stage 1..N-1 (set per step), and
    // the route's SoC-shift bound
    dp_options wo;
    if (opt) wo = *opt;
    else std::memset(&wo, 0, sizeof wo);
    wo.flags = L->timing ? DP_TIMING : DP_GRAPH;
    wo.inst_opt = nullptr;
    const int nwin = std::min(horizon, NR);
    L->win.resize(nwin);
    std::vector<float> init((size_t)route->n_v * route->n_soc * n_t, 0.0f);
    float *dterm = nullptr;
    if ((rc = dev_alloc((void **)&dterm, sizeof(float) * init.size()))) {
        loop_free(L);
        return rc;
    }
    (void)hipMemset(dterm, 0, sizeof(float) * init.size());
    std::vector<int32_t> ps;
    std::vector<double> pc, pr, po;
    for (int N = 1; N <= nwin && !rc; N++) {
        Window &w = L->win[N - 1];
        w.N = N;
        dp_problem_desc d = L->route;
        d.n_stages = N;
        d.t_f = t_f;
        d.n_t = n_t;
        d.theta[4] = 0.0;
        ps.clear();
        pc.assign(N > 1 ? N - 1 : 1, 100.0);
        pr.assign(N > 1 ? N - 1 : 1, 50.0);
        po.assign(N > 1 ? N - 1 : 1, 0.0);
        for (int k = 1; k < N; k++) ps.push_back(k);
        d.n_lights = N - 1;
        d.light_stage = ps.data();
        d.light_cycle = pc.data();
        d.light_red = pr.data();
        d.light_offset = po.data();
        d.light_yellow = nullptr;
        d.terminal_V = dterm;
        d.flags |= DP_TERMINAL_DEVICE;
        rc = build_window_plan(d, fi.soc_shift, &wo, device, &w.p);
        if (!rc) rc = dp_workspace_size(w.p, &bJ, &bpi, &bs);
        if (!rc) rc = dev_alloc(&w.J, bJ);
        if (!rc) rc = dev_alloc(&w.pi, bpi);
        if (!rc) rc = dev_alloc(&w.scr, bs);
        if (!rc) rc = dev_alloc((void **)&w.V0, sizeof(float));
        if (!rc) rc = dev_alloc((void **)&w.u0, sizeof(int16_t));
        if (!rc) rc = dev_alloc((void **)&w.traj, sizeof(double) * 8 * (N + 1));
        if (!rc) rc = dev_alloc((void **)&w.status, sizeof(int32_t) * 2);
        if (!rc) {
            w.term = plan_terminal(w.p);
            dp_instance_info wi;
            rc = dp_instance_info_get(w.p, 0, &wi);
            w.evals = wi.evaluations;
        }
    }
    (void)hipDeviceSynchronize();   // the plans copied the placeholder table at build
    (void)hipFree(dterm);
    if (rc) {
        loop_free(L);
        return rc;
    }
    L->tot.t_abs = route->t0_abs;
    L->tot.v = route->v0;
    L->tot.soc = route->soc0;
    *out = L;
    return DP_OK;
}

int dp_loop_step(dp_loop *L, dp_loop_row *row)
{
    if (!L || !row) return api_fail(DP_EINVAL, "NULL argument");
    const int NR = L->route.n_stages;
    dp_loop_totals &T = L->tot;
    if (L->stopped || T.stage >= NR) return api_fail(DP_ESTATE, "loop: the drive has ended (stage %d)", T.stage);
    hipError_t e = hipSetDevice(L->device);
    if (e != hipSuccess) return api_fail(DP_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    std::memset(row, 0, sizeof *row);
    const int s = T.stage;
    // 1. at rest at a red signal: wait for green
    double tau = 0.0;
    if (T.v == 0.0 && L->light_at[s] >= 0) {
        const int q = L->light_at[s];
        tau = stop_time(L->cyc[q], L->red[q], L->off[q], L->yel[q], L->route.konst[10], 0.0, T.t_abs);
        T.t_abs += tau;
        T.wait_s += tau;
        T.cost += L->route.theta[3] * tau;
    }
    // 2. the horizon s .. s+N in place
    const int N = std::min(L->horizon, NR - s);
    Window &w = L->win[N - 1];
    L->wc.assign(std::max(1, N - 1), 1.0);
    L->wr.assign(std::max(1, N - 1), 0.0);
    L->wo.assign(std::max(1, N - 1), 0.0);
    L->wy.assign(std::max(1, N - 1), 0.0);
    for (int k = 1; k < N; k++) {
        const int q = L->light_at[s + k];
        if (q >= 0) {
            L->wc[k - 1] = L->cyc[q];
            L->wr[k - 1] = L->red[q];
            L->wo[k - 1] = L->off[q];
            L->wy[k - 1] = L->yel[q];
        }
    }
    // 3. its terminal table from the offline values J_{s+N}
    const float *src = (const float *)L->fJ + (size_t)(s + N) * L->fslab;
    int rc = dp_terminal_from_values(src, L->route.n_v, L->route.n_soc, L->route.n_t, L->route.t_f,
                                     T.t_abs - L->route.t0_abs, L->n_t, L->t_f, L->route.konst[13], w.term, L->stream);
    if (!rc)
        rc = plan_set_window(w.p, L->grade.data() + s, L->vmax.data() + s, L->wc.data(), L->wr.data(), L->wo.data(),
                             L->wy.data(), T.t_abs, T.v, T.soc, L->stream);
    // 4. solve, rollout, and the first step back on the host
    if (!rc) rc = dp_solve(w.p, w.J, w.pi, w.scr, w.V0, w.u0, L->stream);
    if (!rc) rc = dp_rollout(w.p, w.pi, w.u0, w.traj, w.status, L->stream);
    if (rc) return rc;
    e = hipMemcpyAsync(L->host, w.traj, sizeof(double) * 16, hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(L->host + 16, w.V0, sizeof(float), hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return api_fail(DP_EDEVICE, "loop: step %d: %s", s, hipGetErrorString(e));
    if ((rc = dp_device_check(w.p, L->stream))) return rc;   // the step's solve is then not used
    if (L->timing) {
        double ms = 0.0;
        int32_t n = 0;
        if ((rc = dp_sweep_time(w.p, &ms, &n))) return rc;
        T.sweep_ms += ms;
        T.sweep_launches += n;
    }
    const double *r0 = L->host, *r1 = L->host + 8;
    float V0;
    std::memcpy(&V0, L->host + 16, sizeof V0);
    row->stage = s;
    row->t_abs = T.t_abs;
    row->v = T.v;
    row->soc = T.soc;
    row->wait_s = tau;
    row->horizon = N;
    row->evaluations = w.evals;
    row->V0 = V0;
    row->u0 = std::isfinite(r0[3]) ? (int32_t)r0[3] : -1;
    row->v1 = r1[0];
    row->soc1 = r1[1];
    row->dt = r1[2];
    row->fuel_g = r1[6];
    row->cost = r1[7];
    T.steps++;
    if (row->u0 < 0 || !(std::isfinite(r1[0]) && std::isfinite(r1[1]) && std::isfinite(r1[2]))) {
        // no admissible control from this state
        L->stopped = true;
        T.status = row->status = DP_EINFEASIBLE;
        return DP_OK;
    }
    // 5. the plant step
    T.fuel_g += r1[6];
    T.cost += r1[7];
    T.stage = s + 1;
    T.v = r1[0];
    T.soc = r1[1];
    T.t_abs += r1[2];
    if (T.stage < NR) {
        if (T.v > L->vmax[T.stage]) row->violations++;
        const int q = L->light_at[T.stage];
        if (T.v > 0.0 && q >= 0 &&
            stop_time(L->cyc[q], L->red[q], L->off[q], L->yel[q], L->route.konst[10], T.v, T.t_abs) > 0.0)
            row->violations++;       // moving through a signal where it has to stop
    }
    T.violations += row->violations;
    if (!(L->route.soc_lo <= T.soc && T.soc <= L->route.soc_hi)) {
        L->stopped = true;
        T.status = row->status = DP_EINFEASIBLE;
    }
    return DP_OK;
}

int dp_loop_get_totals(const dp_loop *L, dp_loop_totals *totals)
{
    if (!L || !totals) return api_fail(DP_EINVAL, "NULL argument");
    *totals = L->tot;
    return DP_OK;
}

void dp_loop_destroy(dp_loop *L) { loop_free(L); }
