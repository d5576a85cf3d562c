/*
 * FP64 CPU oracle for the three-state eco-driving dynamic program.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the tests, the smoke check and the CPU-baseline leg of the benchmark compare
 * the HIP library against.  It shares no code, header, table or constant with
 * the HIP path; the only thing both read is the synthetic instance data.
 *
 * What it computes (Zhu et al., "A GPU Implementation of a Look-Ahead Optimal
 * Controller for Eco-Driving Based on Dynamic Programming", ECC 2021):
 *   - the stage model of Sec. III: speed dynamics Eq. 5a, SoC dynamics Eq. 5b,
 *     time dynamics Eq. 5c, travel time Eq. 2, stage cost Eq. 1 / Eq. 6;
 *   - the constraint set Eq. 7a-d and the signal feasible-time set Eq. 8;
 *   - the backward recursion Eq. 9a-d on uniform grids with trilinear
 *     interpolation of the next-stage cost-to-go, infeasible states and
 *     state-control pairs carrying a large finite cost J_inf (Sec. IV);
 *   - the exact first step at the off-grid initial state (Eq. 6 at x_s);
 *   - a forward rollout of the stored policy and the fixed-policy
 *     derivative of V_0 with respect to theta = (M, CdA, Crr, w_t, w_soc),
 *     both as a backward tangent sweep and as a forward occupancy (adjoint)
 *     sweep.
 * All arithmetic is IEEE double, compiled without fast-math or FMA contraction.
 */
#ifndef ECO_ORACLE_H
#define ECO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t N;              /* horizon stages */
    double ds;              /* distance step [m] */
    const double *grade;    /* [N] road slope (rise/run) of step k -> k+1 */
    const double *vmax;     /* [N+1] route speed limit at stage k */
    int32_t n_lights;
    const int32_t *l_stage; /* [n_lights] signal stages, each in [1, N-1] */
    const double *l_cycle, *l_red, *l_off;
    double t0_abs, v0, soc0;
    double v_lo, v_hi; int32_t n_v;
    double s_lo, s_hi; int32_t n_s;
    double t_f;        int32_t n_t;
    double e_lo, e_hi; int32_t n_e;
    double m_lo, m_hi; int32_t n_m;
    double theta[5];        /* M, CdA, Crr, w_t, w_soc */
    double konst[16];       /* g, rho_air, r_w, i_g, eta_dl, eta_m, C_nom, Voc0, Voc1, R, a_min, a_max, xi_ref, J_inf */
    double fuel[6];         /* q0..q5 */
    const double *terminal_V; /* optional [n_v*n_s*n_t] terminal table, NULL = none */
    int32_t wait_at_red;    /* 1: a stopped vehicle waits out a red phase (Eq. 5c) */
    const double *l_yel;    /* [n_lights] yellow duration Y before red (0 = two phases), or NULL */
} or_inst;

/* Continuous one-step model.  out[] = {v1, dt, cost, acc, P_bat, I_bat, mfuel, q}.
 * Returns 0 if the step is admissible, else a bit set of
 * 1 acceleration bound, 2 speed limit, 4 zero mean speed, 8 battery (D < 0). */
int or_transition(const or_inst *I, int k, double v, double xi, int a, int b, double out[8]);

/* Trilinear interpolation of a slab at index-space coordinates. */
double or_interp(const or_inst *I, const double *J, double rv, double rs, double rt);

/* One backward step: J_k, pi_k (and the second-best value q2) from J_{k+1}. */
void or_stage(const or_inst *I, int k, const double *Jn, double *Jk, int16_t *pik, double *q2k);

/* Value of one node for one control (index a*n_m+b), or the WAIT value for u = -2. */
double or_node_q(const or_inst *I, int k, const double *Jn, int i, int j, int m, int u);

/* One node of the backward step: J_k, pi_k and the second-best value. */
void or_node(const or_inst *I, int k, const double *Jn, int i, int j, int m,
             double *Jout, int32_t *piout, double *q2out);

/* Terminal slab J_N (Eq. 9a). */
void or_terminal(const or_inst *I, double *JN);

/* Exact first step at x0 = (v0, soc0, t = 0): V_0, u_0* and the second best. */
void or_root(const or_inst *I, const double *J1, double *V0, int32_t *u0, double *q2);

/* Full solve; J_all [(N+1)*S], pi_all [N*S], q2_all [N*S] (may be NULL). */
void or_solve(const or_inst *I, double *J_all, int16_t *pi_all, double *q2_all,
              double *V0, int32_t *u0);

/* The rollout's control at an off-grid state (v, xi, t) from one stage's
 * policy slab: among the bracketing nodes of positive interpolation weight
 * whose policy is a control (>= 0), the one of largest weight, equal weights
 * to the lowest linear node index; -1 if none.  Coordinates outside the grid
 * are clamped to it and set *out_of_grid. */
int or_policy_lookup(const or_inst *I, const int16_t *pik, double v, double xi, double t, int32_t *out_of_grid);

/* Forward rollout of the stored policy; traj [(N+1)*8]; returns status
 * (0 ok, -4 no admissible control); *viol counts exact-state violations. */
int or_rollout(const or_inst *I, const int16_t *pi_all, int32_t u0, double *traj, int32_t *viol);

/* Fixed-policy derivative dV_0/dtheta by a backward tangent sweep. */
void or_tangent(const or_inst *I, const double *J_all, const int16_t *pi_all, int32_t u0,
                double grad[5]);

/* The same derivative by a forward occupancy sweep.  Optional diagnostics:
 * rho_sum[N+1] (total occupancy per stage), absorbed[N+1] (mass on nodes at
 * the infeasibility cost, which stops there), exp_cost[N+1] (expected stage
 * cost per stage, expected J_N at N), exp_time (expected total time),
 * exp_socpen (expected terminal (xi - xi_ref)^2), rho_all [(N+1)*S];
 * dgrade[N] (dV_0/dG_k per step); dspat[3 * n_lights] (dV_0 with respect
 * to each signal's offset, red time and cycle, in the order of the
 * instance's signals). */
void or_adjoint(const or_inst *I, const double *J_all, const int16_t *pi_all, int32_t u0,
                double grad[5], double *rho_sum, double *absorbed, double *exp_cost, double *exp_time,
                double *exp_socpen, double *rho_all, double *dgrade, double *dspat);

/* Evaluation counter of a full sweep (dense counting, Sec. IV). */
int64_t or_count_evals(const or_inst *I);

int or_num_threads(void);
void or_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
