/*
 * FP64 CPU oracle for the three-state eco-driving dynamic program.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
 * leg of the benchmark call it; the product path never does.  It shares no
 * code with the HIP library.
 *
 * The code follows the paper's equations (Sec. III) and its serial DP
 * architecture (Sec. IV: a powertrain model per (speed, engine torque, BSG
 * torque) followed by a battery model per SoC node, inside a nested loop over
 * states and controls).  Readings where the paper is silent are stated at the
 * function that applies them.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- grids -- */

/* Uniform grid with inclusive end points: x_i = lo + i*h, h = (hi-lo)/(n-1). */
static double grid_step(double lo, double hi, int n) { return n > 1 ? (hi - lo) / (n - 1) : 0.0; }
static double grid_val(double lo, double hi, int n, int i) { return lo + i * grid_step(lo, hi, n); }

#define K_G 0
#define K_RHO 1
#define K_RW 2
#define K_IG 3
#define K_ETA 4
#define K_ETAM 5
#define K_CNOM 6
#define K_VOC0 7
#define K_VOC1 8
#define K_RBAT 9
#define K_AMIN 10
#define K_AMAX 11
#define K_XIREF 12
#define K_JINF 13
#define K_PENG 14   /* engine power cap [W], 0 = none (Eq. 7e as T_eng <= P/omega(v)) */
#define K_PBSG 15   /* BSG power cap [W], 0 = none (Eq. 7f as |T_bsg| <= P/omega(v)) */

#define T_M 0
#define T_CDA 1
#define T_CRR 2
#define T_WT 3
#define T_WSOC 4

static long slab_size(const or_inst *I) { return (long)I->n_v * I->n_s * I->n_t; }
static long node_index(const or_inst *I, int i, int j, int m) { return ((long)i * I->n_s + j) * I->n_t + m; }

/* ------------------------------------------------------- powertrain model -- */

/* Quantities of one spatial step that depend on (k, v, u) only: the
 * "powertrain model" of the serial architecture (Sec. IV). */
typedef struct {
    double v1;    /* speed at the end of the step, Eq. 5a */
    double acc;   /* mean acceleration over the step */
    double dt;    /* travel time Delta t = Delta d / v_bar, Eq. 2 */
    double cost;  /* stage cost (mf + w_t) * Delta t, Eq. 1 scaled by 1/gamma */
    double mf;    /* fuel rate [g/s] */
    double Pb;    /* battery power demand [W] */
    double q;     /* v^2 + 2 Delta d (F_tr - F_road)/M before the stop clamp */
    double Ftr, Froad;
    double cosa, sina;
    int st;       /* infeasibility bits: 1 accel, 2 speed limit, 4 zero mean speed */
} pt_t;

static void powertrain(const or_inst *I, int k, double v, int a, int b, pt_t *p)
{
    const double *K = I->konst;
    const double M = I->theta[T_M], CdA = I->theta[T_CDA], Crr = I->theta[T_CRR], wt = I->theta[T_WT];
    const double ds = I->ds;
    const double Te = grid_val(I->e_lo, I->e_hi, I->n_e, a);
    const double Tm = grid_val(I->m_lo, I->m_hi, I->n_m, b);
    /* road slope as a fraction: alpha = atan(G), so cos and sin follow algebraically */
    const double G = I->grade[k];
    p->cosa = 1.0 / sqrt(1.0 + G * G);
    p->sina = G * p->cosa;
    /* tractive force of the crank torque through a fixed ratio and driveline efficiency */
    p->Ftr = K[K_ETA] * (Te + Tm) * K[K_IG] / K[K_RW];
    /* road load: rolling resistance + grade + aerodynamic drag at the current speed */
    p->Froad = M * K[K_G] * (Crr * p->cosa + p->sina) + 0.5 * K[K_RHO] * CdA * v * v;
    /* Eq. 5a under a constant force over the step */
    p->q = v * v + 2.0 * ds * (p->Ftr - p->Froad) / M;
    p->st = 0;
    if (p->q > 0.0) {
        p->v1 = sqrt(p->q);
        p->acc = (p->Ftr - p->Froad) / M;
    } else {
        /* the vehicle comes to rest inside the step (the remainder is friction braking) */
        p->v1 = 0.0;
        p->acc = -v * v / (2.0 * ds);
    }
    if (p->acc < K[K_AMIN] || p->acc > K[K_AMAX]) p->st |= 1;       /* Eq. 7d */
    if (p->v1 > I->vmax[k + 1]) p->st |= 2;                          /* Eq. 7a */
    const double vs = v + p->v1;
    if (!(vs > 0.0)) { p->st |= 4; p->dt = INFINITY; }
    else p->dt = 2.0 * ds / vs;                                      /* Eq. 2 */
    /* synthetic fuel map; zero with the engine off (start-stop) */
    double mf = 0.0;
    if (Te != 0.0) {
        const double *q = I->fuel;
        mf = q[0] + q[1] * v + q[2] * Te + q[3] * v * v + q[4] * v * Te + q[5] * Te * Te;
        if (mf < 0.0) mf = 0.0;
    }
    p->mf = mf;
    p->cost = (mf + wt) * p->dt;
    /* BSG mechanical power at the crank speed, motor efficiency by power flow direction */
    const double w = v * K[K_IG] / K[K_RW];
    const double Pm = Tm * w;
    p->Pb = Pm >= 0.0 ? Pm / K[K_ETAM] : Pm * K[K_ETAM];
    /* Eq. 7e-f: speed-dependent torque limits, here the torque a power cap
     * allows at the crank speed of the step's initial speed */
    if (K[K_PENG] > 0.0 && Te * w > K[K_PENG]) p->st |= 16;
    if (K[K_PBSG] > 0.0 && fabs(Tm) * w > K[K_PBSG]) p->st |= 16;
}

/* Zeroth-order equivalent circuit: P_bat = Voc*I - R*I^2, Voc linear in SoC.
 * Returns 0 and the current, or 8 when the demanded power exceeds Voc^2/(4R). */
static int battery_current(const or_inst *I, double Pb, double xi, double *Ib)
{
    const double *K = I->konst;
    const double Voc = K[K_VOC0] + K[K_VOC1] * xi;
    const double D = Voc * Voc - 4.0 * K[K_RBAT] * Pb;
    if (D < 0.0) { *Ib = NAN; return 8; }
    *Ib = 2.0 * Pb / (Voc + sqrt(D));   /* the root (Voc - sqrt(D))/(2R), cancellation free */
    return 0;
}

int or_transition(const or_inst *I, int k, double v, double xi, int a, int b, double out[8])
{
    pt_t p;
    powertrain(I, k, v, a, b, &p);
    double Ib;
    int st = p.st | battery_current(I, p.Pb, xi, &Ib);
    out[0] = p.v1; out[1] = p.dt; out[2] = p.cost; out[3] = p.acc;
    out[4] = p.Pb; out[5] = Ib; out[6] = p.mf; out[7] = p.q;
    return st;
}

/* ------------------------------------------------------------ interpolation -- */

/* One dimension of an index-space coordinate: lower cell c in [0, n-2] and
 * fraction f in [0, 1] with r = c + f, i.e. c = min(floor(r), n-2). */
typedef struct { int c; double f; } cf_t;

static cf_t cf_of(double r, int n)
{
    cf_t x;
    double fl = floor(r);
    x.c = (int)fl;
    if (x.c > n - 2) x.c = n - 2;
    x.f = r - x.c;
    return x;
}

/* The time coordinate of a successor of node m advances by delta cells:
 * r = m + delta, kept as integer cell plus fraction so that an integer
 * advance lands exactly on a node. */
static cf_t cf_shift(int m, double delta, int n)
{
    double fl = floor(delta);
    cf_t x;
    x.c = m + (int)fl;
    x.f = delta - fl;
    if (x.c > n - 2) { x.f = x.f + (x.c - (n - 2)); x.c = n - 2; }
    return x;
}

static int cf_in_range(cf_t x, int n) { return x.c >= 0 && (x.c < n - 2 || (x.c == n - 2 && x.f <= 1.0)) && x.f >= 0.0; }

/* Trilinear interpolation: the sum over the 8 bracketing nodes of weight
 * times value.  Every stored value is finite (an infeasible node holds the
 * large infeasibility cost), so no corner needs special treatment; corners
 * of zero weight are skipped, which also keeps the index inside the grid. */
static double interp_cf(const or_inst *I, const double *J, cf_t v, cf_t s, cf_t t)
{
    double acc = 0.0;
    for (int a = 0; a < 2; a++) {
        double wa = a ? v.f : 1.0 - v.f;
        if (!(wa > 0.0)) continue;
        for (int b = 0; b < 2; b++) {
            double wb = b ? s.f : 1.0 - s.f;
            if (!(wb > 0.0)) continue;
            for (int c = 0; c < 2; c++) {
                double wc = c ? t.f : 1.0 - t.f;
                if (!(wc > 0.0)) continue;
                acc += wa * wb * wc * J[node_index(I, v.c + a, s.c + b, t.c + c)];
            }
        }
    }
    return acc;
}

double or_interp(const or_inst *I, const double *J, double rv, double rs, double rt)
{
    return interp_cf(I, J, cf_of(rv, I->n_v), cf_of(rs, I->n_s), cf_of(rt, I->n_t));
}

/* Partial derivatives of the trilinear interpolant with respect to the three
 * index-space coordinates, inside the cell.  Reading for the measure-zero
 * case of a coordinate exactly on a grid plane (f = 0 or f = 1): that
 * dimension's derivative is taken as 0 (it only occurs where the coordinate
 * itself does not move with theta: no battery current, or a stop). */
static void interp_grad(const or_inst *I, const double *J, cf_t v, cf_t s, cf_t t, double g[3])
{
    const cf_t d[3] = { v, s, t };
    for (int dim = 0; dim < 3; dim++) {
        g[dim] = 0.0;
        if (!(d[dim].f > 0.0 && d[dim].f < 1.0)) continue;
        double acc = 0.0;
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                for (int c = 0; c < 2; c++) {
                    int bits[3] = { a, b, c };
                    double w = 1.0;
                    int skip = 0;
                    for (int e = 0; e < 3; e++) {
                        if (e == dim) continue;
                        double we = bits[e] ? d[e].f : 1.0 - d[e].f;
                        if (!(we > 0.0)) { skip = 1; break; }
                        w *= we;
                    }
                    if (skip) continue;
                    double Jc = J[node_index(I, v.c + a, s.c + b, t.c + c)];
                    acc += (bits[dim] ? 1.0 : -1.0) * w * Jc;
                }
        g[dim] = acc;
    }
}

/* ----------------------------------------------------------- signal lights -- */

static int light_at(const or_inst *I, int k)
{
    for (int L = 0; L < I->n_lights; L++)
        if (I->l_stage[L] == k) return L;
    return -1;
}

/* Signal of stage L at relative time t_rel (Eq. 8, with the yellow phase of
 * Sec. III).  Phase x = (t_abs - offset) mod cycle: red for x in [0, R),
 * yellow for x in [C - Y, C) (the Y seconds before red), green otherwise.
 * Yellow counts as green when the vehicle, crossing at speed v, was within
 * its critical braking distance v^2 / (2 b) of the stop line when yellow
 * began (b = -a_min, the braking limit), i.e. when the time since yellow
 * began is at most v / (2 b); otherwise it has to stop, as in red.  Returns 1
 * when the vehicle has to stop, with *tau the time until green; *phase = x. */
static int must_stop(const or_inst *I, int L, double t_rel, double v, double *tau, double *phase)
{
    const double C = I->l_cycle[L], R = I->l_red[L], Y = I->l_yel ? I->l_yel[L] : 0.0;
    double x = fmod(I->t0_abs + t_rel - I->l_off[L], C);
    if (x < 0.0) x += C;
    *phase = x;
    *tau = 0.0;
    if (x < R) {
        *tau = R - x;
        return 1;
    }
    if (Y > 0.0 && x >= C - Y) {
        const double since = x - (C - Y);
        if (since > v / (2.0 * -I->konst[K_AMIN])) {
            *tau = (C - x) + R;
            return 1;
        }
    }
    return 0;
}

/* 1 when x (a phase from must_stop) lies in the yellow of signal L. */
static int in_yellow(const or_inst *I, int L, double x)
{
    const double C = I->l_cycle[L], R = I->l_red[L], Y = I->l_yel ? I->l_yel[L] : 0.0;
    return !(x < R) && Y > 0.0 && x >= C - Y;
}

/* --------------------------------------------------------- one node, one u -- */

typedef struct {
    double hv, hs, ht;
} steps_t;

static steps_t steps_of(const or_inst *I)
{
    steps_t h;
    h.hv = grid_step(I->v_lo, I->v_hi, I->n_v);
    h.hs = grid_step(I->s_lo, I->s_hi, I->n_s);
    h.ht = grid_step(0.0, I->t_f, I->n_t);
    return h;
}

/* Successor of a state in index space.  rs0 is the SoC coordinate of the
 * current state (j for a node) and m0 the time node (0 for x0).  The speed
 * and SoC parts depend on (k, i, j, u) only; the time part shifts the node
 * index by Delta t / h_t cells. */
typedef struct {
    int ok;
    cf_t v, s, t;
    double Ib;
} succ_t;

static succ_t successor_vs(const or_inst *I, const steps_t *h, const pt_t *p, double xi, double rs0)
{
    succ_t o;
    o.ok = 0;
    if (p->st) return o;
    if (battery_current(I, p->Pb, xi, &o.Ib)) return o;
    double rv = (p->v1 - I->v_lo) / h->hv;
    if (!(rv >= 0.0 && rv <= I->n_v - 1)) return o;
    /* Eq. 5b in index space: the SoC moves by Delta t * I / C_nom */
    double rs = rs0 - (p->dt * o.Ib) / (I->konst[K_CNOM] * h->hs);
    if (!(rs >= 0.0 && rs <= I->n_s - 1)) return o;
    o.v = cf_of(rv, I->n_v);
    o.s = cf_of(rs, I->n_s);
    o.ok = 1;
    return o;
}

static int successor_t(const or_inst *I, const steps_t *h, const pt_t *p, int m0, succ_t *o)
{
    if (!(p->dt / h->ht < I->n_t)) return 0;   /* beyond t_f from any node */
    o->t = cf_shift(m0, p->dt / h->ht, I->n_t);
    return cf_in_range(o->t, I->n_t);
}

static succ_t successor(const or_inst *I, const steps_t *h, const pt_t *p, double xi, double rs0, int m0)
{
    succ_t o = successor_vs(I, h, p, xi, rs0);
    if (o.ok && !successor_t(I, h, p, m0, &o)) o.ok = 0;
    return o;
}

static void control_pair(const or_inst *I, int u, int *a, int *b) { *a = u / I->n_m; *b = u % I->n_m; }

double or_node_q(const or_inst *I, int k, const double *Jn, int i, int j, int m, int u)
{
    const double Jinf = I->konst[K_JINF];
    steps_t h = steps_of(I);
    double v = grid_val(I->v_lo, I->v_hi, I->n_v, i);
    double xi = grid_val(I->s_lo, I->s_hi, I->n_s, j);
    if (u == -2) {
        int L = light_at(I, k);
        double phase, tau;
        if (L < 0 || !must_stop(I, L, grid_val(0.0, I->t_f, I->n_t, m), 0.0, &tau, &phase)) return Jinf;
        cf_t t = cf_shift(m, tau / h.ht, I->n_t);
        if (!cf_in_range(t, I->n_t)) return Jinf;
        cf_t cv = cf_of((double)i, I->n_v), cs = cf_of((double)j, I->n_s);
        return I->theta[T_WT] * tau + interp_cf(I, Jn, cv, cs, t);
    }
    int a, b;
    control_pair(I, u, &a, &b);
    pt_t p;
    powertrain(I, k, v, a, b, &p);
    succ_t sc = successor(I, &h, &p, xi, (double)j, m);
    if (!sc.ok) return Jinf;
    return p.cost + interp_cf(I, Jn, sc.v, sc.s, sc.t);
}

/* One node of Eq. 9b-d: J_k, pi_k and the second-best candidate, from J_{k+1}
 * (the same rule as the stage sweep, evaluated for a single node). */
void or_node(const or_inst *I, int k, const double *Jn, int i, int j, int m,
             double *Jout, int32_t *piout, double *q2out)
{
    const int nu = I->n_e * I->n_m;
    const double Jinf = I->konst[K_JINF];
    const int L = light_at(I, k);
    const double v = grid_val(I->v_lo, I->v_hi, I->n_v, i);
    double best = Jinf, second = Jinf;
    int bu = -1;
    double phase = 0.0, tau = 0.0;
    int red = L >= 0 && must_stop(I, L, grid_val(0.0, I->t_f, I->n_t, m), v, &tau, &phase);
    if (v > I->vmax[k]) {
        /* infeasible node */
    } else if (red) {
        if (v == 0.0 && I->wait_at_red) {
            double val = or_node_q(I, k, Jn, i, j, m, -2);
            if (val < best) { best = val; bu = -2; }
        }
    } else {
        for (int u = 0; u < nu; u++) {
            double Q = or_node_q(I, k, Jn, i, j, m, u);
            if (Q < best) { second = best; best = Q; bu = u; }
            else if (Q < second) second = Q;
        }
    }
    *Jout = best;
    *piout = bu;
    *q2out = second;
}

/* --------------------------------------------------------------- terminal -- */

/* Eq. 9a: J_N = c_T + phi_T.  c_T is a quadratic SoC-deviation penalty (the
 * stand-in for the SoC-neutrality constraint xi_1 = xi_N, Eq. 7) plus an
 * optional user table; phi_T is the speed-limit constraint at stage N.  Like
 * every cost-to-go value it is capped at the infeasibility cost. */
void or_terminal(const or_inst *I, double *JN)
{
    const double wsoc = I->theta[T_WSOC], xref = I->konst[K_XIREF], Jinf = I->konst[K_JINF];
    for (int i = 0; i < I->n_v; i++) {
        double v = grid_val(I->v_lo, I->v_hi, I->n_v, i);
        for (int j = 0; j < I->n_s; j++) {
            double xi = grid_val(I->s_lo, I->s_hi, I->n_s, j);
            double pen = wsoc * (xi - xref) * (xi - xref);
            for (int m = 0; m < I->n_t; m++) {
                long n = node_index(I, i, j, m);
                double val = pen + (I->terminal_V ? I->terminal_V[n] : 0.0);
                JN[n] = (v > I->vmax[I->N] || !(val < Jinf)) ? Jinf : val;
            }
        }
    }
}

/* ------------------------------------------------------------ stage sweep -- */

/* Eq. 9b-d at every node of stage k: the minimum over all control pairs of
 * stage cost plus interpolated J_{k+1} at the successor.  Infeasibility
 * (Sec. IV): a state-control pair that violates a constraint, and a node that
 * does, take the infeasibility cost J_inf, a value orders of magnitude above
 * any stage cost; J_k is the minimum of J_inf and the feasible candidates,
 * so it never exceeds J_inf.  Controls are scanned in ascending
 * u = a*n_m + b with a strict comparison, so the lowest index wins a tie;
 * policy -1 when no control beats J_inf.  Node constraints: speed limit
 * (Eq. 7a) and, at a signal stage, the red-phase exclusion of Eq. 7c/8; a
 * node at zero speed in red instead waits until the phase turns green
 * (Eq. 5c), policy code -2. */
void or_stage(const or_inst *I, int k, const double *Jn, double *Jk, int16_t *pik, double *q2k)
{
    const int nv = I->n_v, ns = I->n_s, nt = I->n_t, nu = I->n_e * I->n_m;
    const steps_t h = steps_of(I);
    const int L = light_at(I, k);
    const double wt = I->theta[T_WT], Jinf = I->konst[K_JINF];

#pragma omp parallel
    {
        pt_t *pt = (pt_t *)malloc(sizeof(pt_t) * nu);
        succ_t *sc = (succ_t *)malloc(sizeof(succ_t) * nu);
#pragma omp for schedule(dynamic, 1)
        for (int ij = 0; ij < nv * ns; ij++) {
            const int i = ij / ns, j = ij % ns;
            const double v = grid_val(I->v_lo, I->v_hi, nv, i);
            const double xi = grid_val(I->s_lo, I->s_hi, ns, j);
            const int speed_bad = v > I->vmax[k];
            for (int u = 0; u < nu; u++) {
                int a, b;
                control_pair(I, u, &a, &b);
                powertrain(I, k, v, a, b, &pt[u]);
                sc[u] = successor_vs(I, &h, &pt[u], xi, (double)j);   /* battery model per SoC node */
            }
            for (int m = 0; m < nt; m++) {
                const long n = node_index(I, i, j, m);
                double best = Jinf, second = Jinf;
                int bu = -1;
                int red = 0;
                double phase = 0.0, tau = 0.0;
                if (L >= 0) red = must_stop(I, L, grid_val(0.0, I->t_f, nt, m), v, &tau, &phase);
                if (speed_bad) {
                    /* infeasible node */
                } else if (red) {
                    if (v == 0.0 && I->wait_at_red) {
                        cf_t t = cf_shift(m, tau / h.ht, nt);
                        if (cf_in_range(t, nt)) {
                            double val = wt * tau + interp_cf(I, Jn, cf_of((double)i, nv), cf_of((double)j, ns), t);
                            if (val < best) { best = val; bu = -2; }
                        }
                    }
                } else {
                    for (int u = 0; u < nu; u++) {
                        if (!sc[u].ok) continue;
                        succ_t s = sc[u];
                        if (!successor_t(I, &h, &pt[u], m, &s)) continue;
                        double Q = pt[u].cost + interp_cf(I, Jn, s.v, s.s, s.t);
                        if (Q < best) { second = best; best = Q; bu = u; }
                        else if (Q < second) second = Q;
                    }
                }
                Jk[n] = best;
                pik[n] = (int16_t)bu;
                if (q2k) q2k[n] = second;
            }
        }
        free(pt);
        free(sc);
    }
}

/* ------------------------------------------------------------------- root -- */

/* Eq. 6 at the actual state x0 = (v0, soc0, t = 0), which need not be a node. */
void or_root(const or_inst *I, const double *J1, double *V0, int32_t *u0, double *q2)
{
    const steps_t h = steps_of(I);
    const int nu = I->n_e * I->n_m;
    double best = I->konst[K_JINF], second = I->konst[K_JINF];
    int bu = -1;
    if (!(I->v0 > I->vmax[0])) {
        const double rs0 = (I->soc0 - I->s_lo) / h.hs;
        for (int u = 0; u < nu; u++) {
            int a, b;
            control_pair(I, u, &a, &b);
            pt_t p;
            powertrain(I, 0, I->v0, a, b, &p);
            succ_t sc = successor(I, &h, &p, I->soc0, rs0, 0);
            if (!sc.ok) continue;
            double Q = p.cost + interp_cf(I, J1, sc.v, sc.s, sc.t);
            if (Q < best) { second = best; best = Q; bu = u; }
            else if (Q < second) second = Q;
        }
    }
    *V0 = best;
    *u0 = bu;
    if (q2) *q2 = second;
}

void or_solve(const or_inst *I, double *J_all, int16_t *pi_all, double *q2_all, double *V0, int32_t *u0)
{
    const long S = slab_size(I);
    or_terminal(I, J_all + (long)I->N * S);
    for (int k = I->N - 1; k >= 0; k--)
        or_stage(I, k, J_all + (long)(k + 1) * S, J_all + (long)k * S, pi_all + (long)k * S,
                 q2_all ? q2_all + (long)k * S : NULL);
    or_root(I, J_all + S, V0, u0, NULL);
}

/* ---------------------------------------------------------------- rollout -- */

/* Control at an off-grid state: among the bracketing nodes of positive
 * interpolation weight whose stored policy is a control (>= 0), the one of
 * largest weight (the nearest node); equal weights go to the lowest linear
 * node index.  Returns -1 if there is none. */
static int policy_lookup(const or_inst *I, const int16_t *pik, double v, double xi, double t, int *out_of_grid)
{
    const steps_t h = steps_of(I);
    double r[3] = { (v - I->v_lo) / h.hv, (xi - I->s_lo) / h.hs, t / h.ht };
    const int n[3] = { I->n_v, I->n_s, I->n_t };
    cf_t c[3];
    for (int d = 0; d < 3; d++) {
        if (r[d] < 0.0) { r[d] = 0.0; *out_of_grid = 1; }
        if (r[d] > n[d] - 1) { r[d] = n[d] - 1; *out_of_grid = 1; }
        c[d] = cf_of(r[d], n[d]);
    }
    double bw = -1.0;
    long bn = -1;
    int bu = -1;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int e = 0; e < 2; e++) {
                double w = (a ? c[0].f : 1.0 - c[0].f) * (b ? c[1].f : 1.0 - c[1].f) * (e ? c[2].f : 1.0 - c[2].f);
                if (!(w > 0.0)) continue;
                long nidx = node_index(I, c[0].c + a, c[1].c + b, c[2].c + e);
                int u = pik[nidx];
                if (u < 0) continue;
                if (w > bw || (w == bw && nidx < bn)) { bw = w; bn = nidx; bu = u; }
            }
    return bu;
}

/* The rollout's control lookup at an off-grid state, for its pin. */
int or_policy_lookup(const or_inst *I, const int16_t *pik, double v, double xi, double t, int32_t *out_of_grid)
{
    int oog = 0;
    const int u = policy_lookup(I, pik, v, xi, t, &oog);
    *out_of_grid = oog;
    return u;
}

/* traj row k = {v, xi, t, u, T_eng, T_mot, fuel so far, cost so far}; the
 * last row's cost includes the terminal cost. */
int or_rollout(const or_inst *I, const int16_t *pi_all, int32_t u0, double *traj, int32_t *viol)
{
    const long S = slab_size(I);
    const steps_t h = steps_of(I);
    const double wt = I->theta[T_WT];
    double v = I->v0, xi = I->soc0, t = 0.0, fuel = 0.0, cost = 0.0;
    int status = 0;
    *viol = 0;
    for (int r = 0; r <= I->N; r++)
        for (int c = 0; c < 8; c++) traj[r * 8 + c] = NAN;
    int k;
    for (k = 0; k < I->N; k++) {
        double *row = traj + k * 8;
        row[0] = v; row[1] = xi; row[2] = t; row[6] = fuel; row[7] = cost;
        int u;
        if (k == 0) {
            u = u0;
            if (v > I->vmax[0]) (*viol)++;
        } else {
            int L = light_at(I, k);
            double phase, tau;
            if (L >= 0 && must_stop(I, L, t, v, &tau, &phase)) {
                if (v == 0.0 && I->wait_at_red) {
                    /* Eq. 5c: wait for green */
                    row[3] = -2.0;
                    t += tau;
                    cost += wt * tau;
                    continue;
                }
                (*viol)++;       /* crossing when it has to stop (red, or yellow past the braking distance) */
            }
            if (v > I->vmax[k]) (*viol)++;
            int oog = 0;
            u = policy_lookup(I, pi_all + (long)k * S, v, xi, t, &oog);
            if (oog) (*viol)++;
        }
        if (u < 0) { status = -4; break; }
        int a, b;
        control_pair(I, u, &a, &b);
        row[3] = u;
        row[4] = grid_val(I->e_lo, I->e_hi, I->n_e, a);
        row[5] = grid_val(I->m_lo, I->m_hi, I->n_m, b);
        pt_t p;
        powertrain(I, k, v, a, b, &p);
        double Ib;
        int bst = battery_current(I, p.Pb, xi, &Ib);
        if ((p.st & 4) || bst) { status = -4; break; }
        if (p.st) (*viol)++;
        fuel += p.mf * p.dt;
        cost += p.cost;
        xi = xi - p.dt * Ib / I->konst[K_CNOM];
        v = p.v1;
        t = t + p.dt;
        if (xi < I->s_lo || xi > I->s_hi || t > I->t_f) (*viol)++;
    }
    if (status == 0) {
        double *row = traj + I->N * 8;
        if (v > I->vmax[I->N]) (*viol)++;
        double pen = I->theta[T_WSOC] * (xi - I->konst[K_XIREF]) * (xi - I->konst[K_XIREF]);
        if (I->terminal_V) {
            double r[3] = { (v - I->v_lo) / h.hv, (xi - I->s_lo) / h.hs, t / h.ht };
            const int n[3] = { I->n_v, I->n_s, I->n_t };
            for (int d = 0; d < 3; d++) r[d] = r[d] < 0 ? 0 : (r[d] > n[d] - 1 ? n[d] - 1 : r[d]);
            pen += or_interp(I, I->terminal_V, r[0], r[1], r[2]);
        }
        cost += pen;
        row[0] = v; row[1] = xi; row[2] = t; row[6] = fuel; row[7] = cost;
    }
    return status;
}

/* ------------------------------------------------------------ derivatives -- */

/* Partial derivatives, with the control held fixed, of the stage cost and of
 * the three successor coordinates with respect to theta.  From Eq. 5a:
 * q = v^2 + 2 dd (F_tr - F_road)/M with F_road = M g (Crr cos + sin) +
 * rho CdA v^2 / 2; v1 = sqrt(q) (0 when clamped); Delta t = 2 dd/(v + v1);
 * the SoC coordinate moves by -Delta t I/(C_nom h_s); the time coordinate by
 * Delta t / h_t; the cost (mf + w_t) Delta t. */
static void step_partials(const or_inst *I, const steps_t *h, double v, const pt_t *p, double Ib,
                          double dc[5], double dr[5][3])
{
    const double M = I->theta[T_M], ds = I->ds, g = I->konst[K_G], rho = I->konst[K_RHO];
    double dq[5] = { 0, 0, 0, 0, 0 };
    dq[T_M] = 2.0 * ds * (-g * (I->theta[T_CRR] * p->cosa + p->sina) / M - (p->Ftr - p->Froad) / (M * M));
    dq[T_CDA] = -ds * rho * v * v / M;
    dq[T_CRR] = -2.0 * ds * g * p->cosa;
    for (int q = 0; q < 5; q++) {
        double dv1 = p->q > 0.0 ? dq[q] / (2.0 * p->v1) : 0.0;
        double vs = v + p->v1;
        double ddt = -2.0 * ds / (vs * vs) * dv1;
        dc[q] = (p->mf + I->theta[T_WT]) * ddt + (q == T_WT ? p->dt : 0.0);
        dr[q][0] = dv1 / h->hv;
        dr[q][1] = -(Ib / (I->konst[K_CNOM] * h->hs)) * ddt;
        dr[q][2] = ddt / h->ht;
    }
}

/* Partial derivatives of the stage cost and of the successor's index
 * coordinates with respect to the grade G of step k (control fixed): G enters
 * only the road load F_road = M g (Crr cos a + sin a) with cos a =
 * 1/sqrt(1 + G^2), sin a = G cos a, so dF_road/dG = M g cos^3 a (1 - Crr G). */
static void grade_partials(const or_inst *I, const steps_t *h, int k, double v, const pt_t *p, double Ib,
                           double *dc, double dr[3])
{
    const double M = I->theta[T_M], ds = I->ds, G = I->grade[k], c = p->cosa;
    const double dFroad = M * I->konst[K_G] * c * c * c * (1.0 - I->theta[T_CRR] * G);
    const double dq = -2.0 * ds * dFroad / M;
    const double dv1 = p->q > 0.0 ? dq / (2.0 * p->v1) : 0.0;
    const double vs = v + p->v1;
    const double ddt = -2.0 * ds / (vs * vs) * dv1;
    *dc = (p->mf + I->theta[T_WT]) * ddt;
    dr[0] = dv1 / h->hv;
    dr[1] = -(Ib / (I->konst[K_CNOM] * h->hs)) * ddt;
    dr[2] = ddt / h->ht;
}

void or_tangent(const or_inst *I, const double *J_all, const int16_t *pi_all, int32_t u0, double grad[5])
{
    const long S = slab_size(I);
    const steps_t h = steps_of(I);
    const int nv = I->n_v, ns = I->n_s, nt = I->n_t;
    double *Dn = (double *)calloc(5 * S, sizeof(double));
    double *Dk = (double *)calloc(5 * S, sizeof(double));
    /* dJ_N/dtheta: only the terminal SoC weight enters (a capped node is constant) */
    const double *JN = J_all + (long)I->N * S;
    for (int i = 0; i < nv; i++)
        for (int j = 0; j < ns; j++) {
            double xi = grid_val(I->s_lo, I->s_hi, ns, j);
            double d = (xi - I->konst[K_XIREF]);
            for (int m = 0; m < nt; m++) {
                long n = node_index(I, i, j, m);
                Dn[T_WSOC * S + n] = JN[n] < I->konst[K_JINF] ? d * d : 0.0;
            }
        }
    for (int k = I->N - 1; k >= 1; k--) {
        const double *Jn = J_all + (long)(k + 1) * S;
        const int16_t *pik = pi_all + (long)k * S;
        const int L = light_at(I, k);
#pragma omp parallel for schedule(dynamic, 4)
        for (int ij = 0; ij < nv * ns; ij++) {
            const int i = ij / ns, j = ij % ns;
            const double v = grid_val(I->v_lo, I->v_hi, nv, i);
            const double xi = grid_val(I->s_lo, I->s_hi, ns, j);
            for (int m = 0; m < nt; m++) {
                const long n = node_index(I, i, j, m);
                const int u = pik[n];
                for (int q = 0; q < 5; q++) Dk[q * S + n] = 0.0;
                if (u == -2) {
                    double phase, tau;
                    must_stop(I, L, grid_val(0.0, I->t_f, nt, m), 0.0, &tau, &phase);
                    cf_t t = cf_shift(m, tau / h.ht, nt);
                    cf_t cv = cf_of((double)i, nv), cs = cf_of((double)j, ns);
                    for (int q = 0; q < 5; q++)
                        Dk[q * S + n] = (q == T_WT ? tau : 0.0) + interp_cf(I, Dn + q * S, cv, cs, t);
                } else if (u >= 0) {
                    int a, b;
                    control_pair(I, u, &a, &b);
                    pt_t p;
                    powertrain(I, k, v, a, b, &p);
                    succ_t sc = successor(I, &h, &p, xi, (double)j, m);
                    if (!sc.ok) continue;
                    double dc[5], dr[5][3], gJ[3];
                    step_partials(I, &h, v, &p, sc.Ib, dc, dr);
                    interp_grad(I, Jn, sc.v, sc.s, sc.t, gJ);
                    for (int q = 0; q < 5; q++)
                        Dk[q * S + n] = dc[q] + dr[q][0] * gJ[0] + dr[q][1] * gJ[1] + dr[q][2] * gJ[2]
                                        + interp_cf(I, Dn + q * S, sc.v, sc.s, sc.t);
                }
            }
        }
        double *tmp = Dn; Dn = Dk; Dk = tmp;
    }
    /* root: Eq. 6 at x0 with the chosen u_0* */
    for (int q = 0; q < 5; q++) grad[q] = NAN;
    if (u0 >= 0) {
        int a, b;
        control_pair(I, u0, &a, &b);
        pt_t p;
        powertrain(I, 0, I->v0, a, b, &p);
        const double rs0 = (I->soc0 - I->s_lo) / h.hs;
        succ_t sc = successor(I, &h, &p, I->soc0, rs0, 0);
        if (sc.ok) {
            double dc[5], dr[5][3], gJ[3];
            step_partials(I, &h, I->v0, &p, sc.Ib, dc, dr);
            interp_grad(I, J_all + S, sc.v, sc.s, sc.t, gJ);
            for (int q = 0; q < 5; q++)
                grad[q] = dc[q] + dr[q][0] * gJ[0] + dr[q][1] * gJ[1] + dr[q][2] * gJ[2]
                          + interp_cf(I, Dn + q * S, sc.v, sc.s, sc.t);
        }
    }
    free(Dn);
    free(Dk);
}

/* Add rho * (trilinear weights) into the next stage's occupancy. */
static void scatter(const or_inst *I, double *rho_next, double rho, cf_t v, cf_t s, cf_t t)
{
    for (int a = 0; a < 2; a++) {
        double wa = a ? v.f : 1.0 - v.f;
        if (!(wa > 0.0)) continue;
        for (int b = 0; b < 2; b++) {
            double wb = b ? s.f : 1.0 - s.f;
            if (!(wb > 0.0)) continue;
            for (int c = 0; c < 2; c++) {
                double wc = c ? t.f : 1.0 - t.f;
                if (!(wc > 0.0)) continue;
                rho_next[node_index(I, v.c + a, s.c + b, t.c + c)] += rho * wa * wb * wc;
            }
        }
    }
}

void or_adjoint(const or_inst *I, const double *J_all, const int16_t *pi_all, int32_t u0,
                double grad[5], double *rho_sum, double *absorbed, double *exp_cost, double *exp_time,
                double *exp_socpen, double *rho_all, double *dgrade, double *dspat)
{
    const long S = slab_size(I);
    const steps_t h = steps_of(I);
    const int nv = I->n_v, ns = I->n_s, nt = I->n_t;
    const double wt = I->theta[T_WT];
    double *rk = (double *)calloc(S, sizeof(double));
    double *rn = (double *)calloc(S, sizeof(double));
    double g[5] = { 0, 0, 0, 0, 0 };
    double etime = 0.0, epen = 0.0;
    for (int q = 0; q < 5; q++) grad[q] = NAN;
    if (rho_sum) for (int k = 0; k <= I->N; k++) rho_sum[k] = 0.0;
    if (absorbed) for (int k = 0; k <= I->N; k++) absorbed[k] = 0.0;
    if (exp_cost) for (int k = 0; k <= I->N; k++) exp_cost[k] = 0.0;
    if (rho_all) memset(rho_all, 0, sizeof(double) * S * (I->N + 1));
    if (dgrade) for (int k = 0; k < I->N; k++) dgrade[k] = NAN;   /* like grad, when x0 has no control */
    if (dspat) for (int q = 0; q < 3 * I->n_lights; q++) dspat[q] = NAN;
    if (u0 < 0) goto done;
    if (dspat) for (int q = 0; q < 3 * I->n_lights; q++) dspat[q] = 0.0;
    {
        /* the root step from x0 puts unit mass on the bracketing nodes of stage 1 */
        int a, b;
        control_pair(I, u0, &a, &b);
        pt_t p;
        powertrain(I, 0, I->v0, a, b, &p);
        const double rs0 = (I->soc0 - I->s_lo) / h.hs;
        succ_t sc = successor(I, &h, &p, I->soc0, rs0, 0);
        if (!sc.ok) goto done;
        double dc[5], dr[5][3], gJ[3];
        step_partials(I, &h, I->v0, &p, sc.Ib, dc, dr);
        interp_grad(I, J_all + S, sc.v, sc.s, sc.t, gJ);
        for (int q = 0; q < 5; q++) g[q] += dc[q] + dr[q][0] * gJ[0] + dr[q][1] * gJ[1] + dr[q][2] * gJ[2];
        if (dgrade) {
            double dcg, drg[3];
            grade_partials(I, &h, 0, I->v0, &p, sc.Ib, &dcg, drg);
            for (int k = 0; k < I->N; k++) dgrade[k] = 0.0;
            dgrade[0] = dcg + drg[0] * gJ[0] + drg[1] * gJ[1] + drg[2] * gJ[2];
        }
        if (rho_sum) rho_sum[0] = 1.0;
        if (exp_cost) exp_cost[0] = p.cost;
        etime += p.dt;
        scatter(I, rk, 1.0, sc.v, sc.s, sc.t);
    }
    for (int k = 1; k < I->N; k++) {
        const double *Jn = J_all + (long)(k + 1) * S;
        const int16_t *pik = pi_all + (long)k * S;
        const int L = light_at(I, k);
        memset(rn, 0, sizeof(double) * S);
        if (rho_all) memcpy(rho_all + (long)k * S, rk, sizeof(double) * S);
        for (int i = 0; i < nv; i++) {
            const double v = grid_val(I->v_lo, I->v_hi, nv, i);
            for (int j = 0; j < ns; j++) {
                const double xi = grid_val(I->s_lo, I->s_hi, ns, j);
                for (int m = 0; m < nt; m++) {
                    const long n = node_index(I, i, j, m);
                    const double r = rk[n];
                    if (!(r > 0.0)) continue;
                    if (rho_sum) rho_sum[k] += r;
                    const int u = pik[n];
                    if (u == -2) {
                        double phase, tau;
                        must_stop(I, L, grid_val(0.0, I->t_f, nt, m), 0.0, &tau, &phase);
                        cf_t t = cf_shift(m, tau / h.ht, nt);
                        g[T_WT] += r * tau;
                        etime += r * tau;
                        if (exp_cost) exp_cost[k] += r * wt * tau;
                        if (dspat) {
                            /* signal timing (Eq. 5c, Eq. 8): the wait value
                             * w_t tau + J_{k+1}(t_m + tau) moves with tau =
                             * R - phase in red and tau = C - phase + R in
                             * yellow, and phase = t - O - n C (n whole
                             * cycles), so dtau/dO = dtau/dR = 1 and dtau/dC =
                             * n (red) or n + 1 (yellow).  The red and yellow
                             * masks are constant between switching instants:
                             * their derivative is zero. */
                            double gJ[3];
                            interp_grad(I, Jn, cf_of((double)i, nv), cf_of((double)j, ns), t, gJ);
                            const double dval = wt + gJ[2] / h.ht;
                            const double t_abs = I->t0_abs + grid_val(0.0, I->t_f, nt, m);
                            const double ncyc = nearbyint((t_abs - I->l_off[L] - phase) / I->l_cycle[L]);
                            dspat[3 * L + 0] += r * dval;
                            dspat[3 * L + 1] += r * dval;
                            dspat[3 * L + 2] += r * dval * (ncyc + (in_yellow(I, L, phase) ? 1.0 : 0.0));
                        }
                        scatter(I, rn, r, cf_of((double)i, nv), cf_of((double)j, ns), t);
                    } else if (u >= 0) {
                        int a, b;
                        control_pair(I, u, &a, &b);
                        pt_t p;
                        powertrain(I, k, v, a, b, &p);
                        succ_t sc = successor(I, &h, &p, xi, (double)j, m);
                        if (!sc.ok) continue;
                        double dc[5], dr[5][3], gJ[3];
                        step_partials(I, &h, v, &p, sc.Ib, dc, dr);
                        interp_grad(I, Jn, sc.v, sc.s, sc.t, gJ);
                        for (int q = 0; q < 5; q++)
                            g[q] += r * (dc[q] + dr[q][0] * gJ[0] + dr[q][1] * gJ[1] + dr[q][2] * gJ[2]);
                        if (dgrade) {
                            double dcg, drg[3];
                            grade_partials(I, &h, k, v, &p, sc.Ib, &dcg, drg);
                            dgrade[k] += r * (dcg + drg[0] * gJ[0] + drg[1] * gJ[1] + drg[2] * gJ[2]);
                        }
                        etime += r * p.dt;
                        if (exp_cost) exp_cost[k] += r * p.cost;
                        scatter(I, rn, r, sc.v, sc.s, sc.t);
                    } else {
                        /* J_k is the constant infeasibility cost here: the mass stops */
                        if (absorbed) absorbed[k] += r;
                        if (exp_cost) exp_cost[k] += r * I->konst[K_JINF];
                    }
                }
            }
        }
        double *tmp = rk; rk = rn; rn = tmp;
    }
    {
        const double *JN = J_all + (long)I->N * S;
        if (rho_all) memcpy(rho_all + (long)I->N * S, rk, sizeof(double) * S);
        for (int i = 0; i < nv; i++)
            for (int j = 0; j < ns; j++) {
                const double xi = grid_val(I->s_lo, I->s_hi, ns, j);
                const double d2 = (xi - I->konst[K_XIREF]) * (xi - I->konst[K_XIREF]);
                for (int m = 0; m < nt; m++) {
                    const long n = node_index(I, i, j, m);
                    const double r = rk[n];
                    if (!(r > 0.0)) continue;
                    if (rho_sum) rho_sum[I->N] += r;
                    if (JN[n] < I->konst[K_JINF]) g[T_WSOC] += r * d2;
                    else if (absorbed) absorbed[I->N] += r;
                    epen += r * d2;
                    if (exp_cost) exp_cost[I->N] += r * JN[n];
                }
            }
    }
    for (int q = 0; q < 5; q++) grad[q] = g[q];
done:
    if (exp_time) *exp_time = etime;
    if (exp_socpen) *exp_socpen = epen;
    free(rk);
    free(rn);
}

int64_t or_count_evals(const or_inst *I)
{
    /* one evaluation per (node, control) pair visited by the 5-level loop */
    int64_t n = 0;
    for (int k = 0; k < I->N; k++)
        for (int i = 0; i < I->n_v; i++)
            for (int j = 0; j < I->n_s; j++)
                n += (int64_t)I->n_t * I->n_e * I->n_m;
    return n;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (timing on one core); n < 1 keeps
 * the current setting. */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
