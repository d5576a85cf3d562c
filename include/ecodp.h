/*
 * ecodp.h - C ABI of the MI355X (gfx950) dynamic-programming eco-driving solver.
 *
 * The library solves the receding-horizon optimal control problem of Zhu et
 * al., "A GPU Implementation of a Look-Ahead Optimal Controller for Eco-Driving
 * Based on Dynamic Programming" (ECC 2021), Sec. III: states x = (speed v,
 * battery SoC xi, travel time t) (Eq. 4a), controls u = (engine torque,
 * BSG/motor torque) (Eq. 4b), dynamics Eq. 5a-c, stage cost Eq. 1 / Eq. 6,
 * constraints Eq. 7a-d and the signal feasible-time set Eq. 8, by the backward
 * recursion Eq. 9a-d on uniform grids with trilinear interpolation of the
 * next-stage cost-to-go.  Infeasible states and state-control pairs carry the
 * large finite cost J_inf of Sec. IV (konst[13]); every stored cost-to-go is
 * at most J_inf.
 *
 * Conventions for every entry point:
 *  - All functions return an int status: DP_OK (0) or a negative DP_E* code.
 *    Nothing throws across the ABI.  dp_last_error() gives a message for the
 *    last failure on the calling thread.
 *  - Argument validation errors are returned synchronously, before any work
 *    is enqueued.  Work is enqueued asynchronously on the HIP stream given as
 *    `stream` (a hipStream_t; NULL = the default stream); device faults show up
 *    as DP_EDEVICE at a later call or at stream synchronisation.
 *  - Buffers named *_dev and the J / pi / scratch buffers are DEVICE memory
 *    owned by the caller, borrowed until the enqueued work completes.  Sizes
 *    come from dp_workspace_size(); per-instance offsets from dp_instance_info().
 *    The plan owns host metadata, a small device block of parameters and job
 *    tables, a few streams and events of its own (work it puts on them is
 *    joined back into the caller's stream before the call's later work), a
 *    recorded graph (DP_GRAPH) and a small pinned staging buffer
 *    (dp_set_state); dp_destroy releases them.
 *  - A plan must not be used from two host threads at once, and its calls on
 *    different streams must not overlap (they share the scratch buffer).
 *
 * Data layouts (all row-major, travel time fastest):
 *  - value slab J_k: float [n_v][n_soc][n_t]; policy slab pi_k: int16 [n_v][n_soc][n_t]
 *    holding u = a*n_tm + b (a engine-torque index, b motor-torque index),
 *    -1 = no control beats J_inf, -2 = wait for green at a red signal (Eq. 5c).
 *  - J buffer, per instance: (N+1) slabs J_0..J_N when DP_STORE_ALL_V is set,
 *    else 2 slabs used alternately (J_k in slab k % 2; J_0 ends in slab 0).
 *  - pi buffer, per instance: N slabs pi_0..pi_{N-1}.
 */
#ifndef ECODP_H
#define ECODP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DP_OK = 0,
    DP_EINVAL = -1,        /* invalid argument (NaN, bad grid, bad index, ...) */
    DP_ENOMEM = -2,        /* host or device allocation failed */
    DP_EDEVICE = -3,       /* no usable device, or a HIP runtime error */
    DP_EINFEASIBLE = -4,   /* rollout: no admissible control from the current state */
    DP_ESTATE = -5,        /* call out of order (e.g. adjoint without stored values) */
    DP_EUNSUPPORTED = -6   /* size or option outside what this build supports */
};

/* dp_problem_desc.flags */
#define DP_WAIT_AT_RED 1u      /* a stopped vehicle at a red signal waits for green (Eq. 5c) */
#define DP_TERMINAL_DEVICE 2u  /* terminal_V is a device pointer, copied device to device at
                                  dp_build_problem on the null stream (work that wrote it on a
                                  blocking stream has finished by then); else a host pointer */

/* dp_options.flags */
#define DP_STORE_ALL_V 1u      /* keep J_0..J_N (needed by dp_adjoint and for inspection) */
#define DP_TIMING 2u           /* time every state-sweep launch with HIP events */
#define DP_GRAPH 4u            /* dp_solve records its launches once into a HIP graph and replays it;
                                  the graph is recorded again when the buffers change.  Not with
                                  DP_TIMING. */
#define DP_ROUNDS 8u           /* a plan of several instances solves in rounds of launches (round r:
                                  stage N_b-1-r of every instance b) instead of the persistent sweep */
#define DP_STALL_TEST 16u      /* test hook of the persistent sweep's bounded wait: the first job of
                                  every queue waits for a count that is never reached, gives up after
                                  1000 polls and sets the device error word (dp_device_check reports
                                  DP_EDEVICE); the solve's results are then not valid */
#define DP_ADJOINT_WIDE 32u    /* the adjoint's stage kernel takes 2048-node chunks whatever the grid
                                  (chosen by itself on grids of at least 4 Mi nodes per stage); the
                                  gradient is the same up to the order of FP64 additions */

/* One receding-horizon problem (Eq. 6-8).  Host pointers; copied at build. */
typedef struct {
    int32_t n_stages;          /* N >= 1 steps of ds metres                                     */
    double ds;                 /* distance step Delta d [m] (Eq. 2)                              */
    const double *grade;       /* [N] slope (rise/run) of step k -> k+1                          */
    const double *v_max;       /* [N+1] route speed limit at stage k [m/s] (Eq. 7a); NULL = v_hi  */
    int32_t n_lights;          /* signals on the horizon                                          */
    const int32_t *light_stage;/* [n_lights] distinct stages in [1, N-1]                           */
    const double *light_cycle; /* [n_lights] cycle C [s]                                           */
    const double *light_red;   /* [n_lights] red duration R in (0, C] [s]                          */
    const double *light_offset;/* [n_lights] offset O [s]: red iff (t_abs - O) mod C in [0, R)     */
    double t0_abs;             /* absolute clock at the horizon start [s]                          */
    double v0, soc0;           /* initial state x0 = (v0, soc0, t = 0), need not be a grid node    */
    double v_lo, v_hi; int32_t n_v;      /* speed grid, inclusive, v_lo >= 0, n_v >= 2             */
    double soc_lo, soc_hi; int32_t n_soc;/* SoC grid, n_soc >= 2                                   */
    double t_f; int32_t n_t;             /* travel-time grid [0, t_f], n_t >= 2                    */
    double te_lo, te_hi; int32_t n_te;   /* engine torque grid [Nm], n_te >= 1 (lo == hi if 1)     */
    double tm_lo, tm_hi; int32_t n_tm;   /* BSG torque grid [Nm], n_tm >= 1                         */
    double theta[5];           /* M [kg], CdA [m^2], Crr, w_t [g/s], w_soc [g]                     */
    double konst[16];          /* g, rho_air, r_w, i_g, eta_dl, eta_m, C_nom [C], Voc0, Voc1 [V],
                                  R [ohm], a_min, a_max [m/s^2], xi_ref, J_inf, P_eng_max [W],
                                  P_bsg_max [W]: the speed-dependent torque limits of Eq. 7e-f as
                                  T_eng <= P_eng_max / omega(v), |T_bsg| <= P_bsg_max / omega(v) at
                                  the crank speed omega of the step's initial speed (0 = no cap) */
    double fuel[6];            /* fuel rate q0 + q1 v + q2 T + q3 v^2 + q4 v T + q5 T^2 [g/s], T > 0 */
    const float *terminal_V;   /* optional [n_v][n_soc][n_t] added to the terminal cost; NULL = none
                                  (host memory, or device memory with DP_TERMINAL_DEVICE).  Values
                                  must not be negative (costs are not; the sweep relies on it): a
                                  negative host value fails the build with DP_EINVAL, a negative
                                  device value sets the device error word (dp_device_check); NaN
                                  makes the node J_inf                                             */
    uint32_t flags;            /* DP_WAIT_AT_RED, DP_TERMINAL_DEVICE */
    const double *light_yellow;/* [n_lights] yellow duration Y >= 0 before red, Y + R <= C: yellow iff
                                  (t_abs - O) mod C in [C - Y, C) (three-phase signals, Sec. III), or
                                  NULL = none.  A vehicle crossing at speed v in yellow must stop, as
                                  in red, when the time since yellow began exceeds v / (2 b), b =
                                  -a_min (it was beyond its critical braking distance v^2 / (2 b)
                                  when yellow began); else yellow counts as green.  Needs a_min < 0. */
} dp_problem_desc;

typedef struct {
    uint32_t flags;            /* DP_STORE_ALL_V | DP_TIMING | DP_GRAPH                            */
    int32_t kernel;            /* state-sweep variant: 0 automatic, 1 simple per-node, 2 grouped LDS */
    int32_t tile[4];           /* 0 = automatic; tile[0] = SoC rows per workgroup (4, 8, 16),
                                  tile[1] = workgroups sharing one node tile (control slices, <= 16),
                                  tile[2] = resident sweep workgroups per CU (capped by LDS), tile[3] = 0 */
    const int32_t *inst_opt;   /* optional [n_inst][4] per-instance {kernel, tile[0], tile[1], tile[2]},
                                  same meanings, 0 = the plan-wide value; NULL = none (e.g. the
                                  choices of an autotuner for each problem shape)                   */
} dp_options;

typedef struct dp_plan dp_plan;

typedef struct {
    int32_t n_stages, n_v, n_soc, n_t, n_u;
    size_t J_offset;           /* byte offset of the instance's value slabs in the J buffer        */
    size_t pi_offset;          /* byte offset of its policy slabs in the pi buffer                 */
    size_t traj_offset;        /* element (double) offset of its rollout rows in traj_dev          */
    size_t slab_elems;         /* n_v * n_soc * n_t                                                */
    int64_t evaluations;       /* N * slab_elems * n_u (dense state-control evaluations)           */
    int32_t sweep_kernel;      /* state-sweep variant chosen: 1 simple per-node, 2 grouped LDS      */
    int32_t sweep_tile;        /* SoC rows per workgroup (grouped sweep)                           */
    int32_t sweep_split;       /* control slices per node tile (grouped sweep)                     */
    int32_t sweep_grid;        /* persistent workgroups of one grouped-sweep launch                */
    int32_t soc_shift;         /* host bound H on the SoC-cell shift of one step                   */
    int32_t sweep_persistent;  /* 1: solved by the plan's persistent multi-instance sweep (then
                                  sweep_split is 1 and sweep_grid the workgroups of its kernel class) */
} dp_instance_info;

/* Validate n_inst problem descriptions, precompute host-side tables in FP64
 * (grade trigonometry, speed limits, signal red masks and wait times) and
 * upload them to `device`.  On success *out owns the plan (dp_destroy). */
int dp_build_problem(const dp_problem_desc *desc, int32_t n_inst, const dp_options *opt,
                     int device, dp_plan **out);

/* Bytes the caller must provide for the J, pi and scratch buffers of dp_solve,
 * dp_rollout and dp_adjoint (all instances of the plan). */
int dp_workspace_size(const dp_plan *p, size_t *bytes_J, size_t *bytes_pi, size_t *bytes_scratch);

/* Sizes, buffer offsets and the state-sweep configuration chosen for instance
 * `inst` (0 <= inst < n_inst). */
int dp_instance_info_get(const dp_plan *p, int32_t inst, dp_instance_info *info);

/* Backward recursion Eq. 9a-d for every instance: J_N (Eq. 9a), then for
 * k = N-1..0 the stage table and the state sweep (min and argmin over all
 * controls at every node), then the exact first step at x0 (Eq. 6):
 * V0_dev[inst] = min(J_inf, min_u c + interp J_1), u0_dev[inst] = argmin or -1.
 * A plan of several instances on the grouped sweep runs one persistent launch
 * per kernel class (SoC tile and workgroup size): each instance is served by
 * the workgroups of one XCD, whose stage-k work waits (bounded) on a device
 * counter of the instance's finished stage-(k+1) work; a wait that gives up
 * sets the device error word (dp_device_check).  With DP_ROUNDS, or when the
 * persistent sweep does not fit, the instances run in rounds of one stage each
 * (round r: stage N_b-1-r of every instance b with N_b > r).  Either way each
 * instance's results are bit for bit those of a plan holding it alone.  Among exactly equal candidates the
 * grouped sweep keeps the first in its visit order (successor speed cell,
 * then control index); the simple sweep keeps the lowest control index.
 * With DP_GRAPH the launches are recorded into a HIP graph on the first call
 * (and again whenever the buffers differ from the recorded ones) and the
 * graph is replayed on `stream`. */
int dp_solve(dp_plan *p, void *J, void *pi, void *scratch, float *V0_dev, int16_t *u0_dev,
             void *stream);

/* dp_solve without a scratch argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The kernels use a
 * scratch array of DP_STATIC_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends; a plan whose
 * dp_workspace_size() scratch exceeds it gets DP_EUNSUPPORTED (nothing
 * enqueued).  The launches are those of dp_solve, enqueued eagerly on
 * `stream` (a DP_GRAPH plan's graph is neither recorded nor replayed, and
 * no DP_TIMING events are recorded); the results are bit for bit those of
 * dp_solve.  Every call on one device shares that array, and it keeps the
 * last call's contents (the solve clears what must start at zero): calls
 * that overlap on one device, from any plan or stream, race and must be
 * ordered by the caller.  Later dp_adjoint / dp_stage calls take their own
 * scratch buffer as before. */
#define DP_STATIC_SCRATCH_BYTES (64ull << 20)
int dp_solve_static(dp_plan *p, void *J, void *pi, float *V0_dev, int16_t *u0_dev, void *stream);

/* One backward step k of instance `inst` from a caller-provided J_{k+1} slab
 * (device float [n_v][n_soc][n_t], values >= 0 as every value slab of a
 * solve; a negative value gives unspecified minima) into J_out / pi_out
 * (device slabs, not aliasing J_next), with the configuration dp_solve uses
 * for that stage; the stage tables are rebuilt in `scratch`. */
int dp_stage(dp_plan *p, int32_t inst, int32_t k, const float *J_next, float *J_out,
             int16_t *pi_out, void *scratch, void *stream);

/* Receding horizon (Eq. 6): move instance `inst` to a new initial state
 * x0 = (v0, soc0, t = 0) at absolute clock t0_abs without rebuilding the plan.
 * The signal tables (Eq. 8 red sets and the Eq. 5c waits) are recomputed on
 * the host in FP64 and uploaded with the parameter block through plan-owned
 * pinned memory, ordered on `stream` before later work; a solve recorded with
 * DP_GRAPH picks the new state up on its next replay.  v0 >= 0 and soc0 inside
 * the SoC grid, all finite, else DP_EINVAL with nothing changed.  The stored
 * values and policy are stale afterwards (dp_adjoint needs a new dp_solve). */
int dp_set_state(dp_plan *p, int32_t inst, double v0, double soc0, double t0_abs, void *stream);

/* Closed-loop receding horizon (Sec. III after Eq. 9, Sec. V): the terminal
 * cost of a horizon is taken from the value function of an offline DP over
 * the whole route.  This builds the terminal table of a horizon that starts
 * at clock t_shift of that longer solve, from one of its value slabs:
 * src: device float [n_v][n_soc][n_t_src] on the time grid [0, t_f_src];
 * dst: device float [n_v][n_soc][n_t_dst] on the time grid [0, t_f_dst], the
 * speed and SoC grids shared.  Node m of dst is the linear interpolation in
 * time of src at t = t_shift + m t_f_dst / (n_t_dst - 1), computed in FP64
 * and rounded once to FP32, capped at J_inf; a t past t_f_src gives J_inf.
 * Pass dst as terminal_V (with DP_TERMINAL_DEVICE and w_soc = 0) of the
 * horizon's problem.  n_v, n_soc >= 1, n_t_src, n_t_dst >= 2, t_f_src,
 * t_f_dst > 0, t_shift >= 0, J_inf > 0, all finite, pointers non-NULL, else
 * DP_EINVAL.  Enqueued on `stream`; src and dst must not overlap; the caller
 * owns both. */
int dp_terminal_from_values(const float *src, int32_t n_v, int32_t n_soc, int32_t n_t_src,
                            double t_f_src, double t_shift, int32_t n_t_dst, double t_f_dst,
                            double J_inf, float *dst, void *stream);

/* The closed-loop receding-horizon controller (Sec. V, Sec. III after Eq. 9)
 * along one route, kept in the library.  dp_loop_create copies the route
 * (n_stages N_route, grade, speed limits, signals, x0 and clock t0_abs, the
 * route's own terminal cost) and solves it once over the whole route
 * (DP_STORE_ALL_V): the offline DP whose value slabs give every horizon its
 * terminal cost.  It then builds one plan per horizon length
 * N = 1 .. min(horizon, N_route), each on the time grid [0, t_f] x n_t with
 * the route's speed, SoC and control grids and w_soc = 0, kept for the whole
 * drive.  opt: kernel and tile choices for the horizon plans (NULL = automatic);
 * of its flags only DP_TIMING is used (the summed sweep time of every step in
 * dp_loop_totals; without it the horizon solves are recorded as HIP graphs
 * and replayed).  All device memory is allocated here, none per step.
 *
 * dp_loop_step drives one route stage s from the state (v, soc, t_abs):
 *   1. a vehicle at rest (v == 0) at the stop line of a signal of stage s
 *      that shows red (Eq. 8: red iff (t_abs - O) mod C < R) waits for green
 *      (Eq. 5c): t_abs and the trip's waiting time grow by the rest of the red
 *      phase and the trip cost by w_t times it;
 *   2. the horizon of the next N = min(horizon, N_route - s) steps (grades
 *      s..s+N-1, limits s..s+N, the signals strictly inside, re-indexed from
 *      s) is written into the kept plan of length N in place, with x0 =
 *      (v, soc) and clock t_abs;
 *   3. its terminal table is the offline value slab J_{s+N} shifted by
 *      t_abs - t0_abs (dp_terminal_from_values);
 *   4. dp_solve and dp_rollout; the rollout's first step, under u_0*, is the
 *      plant step (exact FP64 dynamics, Eq. 1-2, 5a-b);
 *   5. the vehicle moves to stage s+1: (v, soc) from that step, t_abs + dt;
 *      fuel and cost of the step are added to the trip; arriving above the
 *      speed limit of stage s+1, or moving (v > 0) at a signal of stage s+1
 *      during red, counts one violation each; a SoC off the grid, no
 *      admissible control (u_0* = -1) or a non-finite step stops the loop
 *      with status DP_EINFEASIBLE.
 * The row describes the step; its status is the loop's.  After the last
 * stage, or once stopped, dp_loop_step returns DP_ESTATE.  Each step reads
 * the horizon plan's device error word (dp_device_check) after its solve and
 * returns DP_EDEVICE without moving the vehicle when a kernel set it;
 * dp_loop_create checks the full-route solve the same way.  A loop must not
 * be used from two host threads at once. */
typedef struct dp_loop dp_loop;

typedef struct {
    int32_t stage;             /* route stage s of the step                                         */
    double t_abs, v, soc;      /* clock [s] and state at the solve (after any wait)                */
    double wait_s;             /* seconds waited at the stop line before the solve                 */
    int32_t horizon;           /* N of the step's horizon                                          */
    int64_t evaluations;       /* state-control evaluations of its solve (N n_v n_soc n_t n_u)     */
    float V0;                  /* V_0 of the horizon                                               */
    int32_t u0;                /* applied control u_0* (-1: none)                                  */
    double v1, soc1, dt;       /* the plant step under u_0*                                        */
    double fuel_g, cost;       /* fuel [g] and cost of the step                                    */
    int32_t violations;        /* violations counted at arrival at stage s+1 (0, 1 or 2)           */
    int32_t status;            /* DP_OK, or DP_EINFEASIBLE when the loop stopped at this step       */
} dp_loop_row;

typedef struct {
    int32_t stage;             /* route stage of the vehicle                                        */
    double t_abs, v, soc;      /* current clock and state                                           */
    double fuel_g, cost, wait_s;
    int32_t violations;
    int32_t status;            /* DP_OK, or DP_EINFEASIBLE once stopped                             */
    int32_t steps;             /* steps driven                                                      */
    double offline_ms;         /* host time of dp_loop_create's full-route solve                    */
    double sweep_ms;           /* with DP_TIMING: summed state-sweep launch time of all steps       */
    int32_t sweep_launches;
} dp_loop_totals;

int dp_loop_create(const dp_problem_desc *route, int32_t horizon, double t_f, int32_t n_t,
                   const dp_options *opt, int32_t device, dp_loop **out);
int dp_loop_step(dp_loop *loop, dp_loop_row *row);
int dp_loop_get_totals(const dp_loop *loop, dp_loop_totals *totals);
void dp_loop_destroy(dp_loop *loop);

/* Forward rollout of the stored policy from x0 with exact FP64 dynamics.
 * traj_dev: double rows [v, xi, t, u, T_eng, T_mot, fuel_g, cost] for stages
 * 0..N of every instance (offset dp_instance_info.traj_offset); the last row's
 * cost includes the terminal cost.  status_dev[2*inst] = DP_OK or
 * DP_EINFEASIBLE, status_dev[2*inst+1] = count of exact-state constraint
 * violations (red crossing, speed limit, leaving the grid). */
int dp_rollout(dp_plan *p, const void *pi, const int16_t *u0_dev, double *traj_dev,
               int32_t *status_dev, void *stream);

/* Fixed-policy derivative dV_0/dtheta, theta = (M, CdA, Crr, w_t, w_soc), by
 * a forward sweep of the occupancy measure (the transpose of the
 * interpolation) over the stored J_0..J_N and pi.  Requires DP_STORE_ALL_V.
 * grad_dev: double [n_inst][5]. */
int dp_adjoint(dp_plan *p, const void *J, const void *pi, const int16_t *u0_dev,
               void *scratch, double *grad_dev, void *stream);

/* dp_adjoint plus the sensitivity of V_0 to the grade of every step (a
 * route parameter per step, Eq. 5a through the road load): dgrade_dev: double
 * [sum over instances of N], instance b at the offset of the N of the
 * instances before it, dgrade[k] = dV_0/dG_k with the policy fixed.  G_k
 * enters only the road load of step k, like C_rr, so dV_0/dG_k is
 * cos a_k (cos a_k - C_rr sin a_k) times step k's share of dV_0/dC_rr; the
 * shares are kept per step in the scratch buffer.  Not a number where x0 has
 * no admissible control (as grad_dev). */
int dp_adjoint_grade(dp_plan *p, const void *J, const void *pi, const int16_t *u0_dev,
                     void *scratch, double *grad_dev, double *dgrade_dev, void *stream);

/* dp_adjoint plus the sensitivity of V_0 to the timing of every signal
 * (Eq. 8: offset O, red time R, cycle C; Eq. 5c: a vehicle stopped at a red
 * signal waits tau = R - phase, with phase = t_abs - O - n C for n whole
 * cycles).  dspat_dev: double [sum over instances of 3 n_lights], instance b
 * at the offset of the 3 n_lights of the instances before it, signal L of
 * the instance (in the order of its light arrays) at 3 L + (0, 1, 2) =
 * dV_0/d(O, R, C) with the policy fixed.  Only the wait moves with the
 * timing: a wait node adds rho (w_t + dJ_{k+1}/dt) times dtau, with
 * dtau/dO = dtau/dR = 1 and dtau/dC = n; the red flags of the time nodes are
 * constant between switching instants and add nothing.  The wait sums are
 * kept per signal in the scratch buffer.  Not a number where x0 has no
 * admissible control (as grad_dev); DP_EINVAL if dspat_dev is NULL. */
int dp_adjoint_spat(dp_plan *p, const void *J, const void *pi, const int16_t *u0_dev,
                    void *scratch, double *grad_dev, double *dspat_dev, void *stream);

/* State-control evaluations the state sweep executed for each instance
 * since the start of the last dp_solve (plus those of dp_stage calls made
 * after it): counts[inst] for every instance of the plan, a host array.
 * The grouped sweep counts, per (speed node, SoC tile), the controls it
 * visits with at least one admissible successor row in the tile, times the
 * tile's rows and the time nodes (nodes above the stage's speed limit and
 * controls infeasible for the whole row are skipped, Eq. 7a-d); the simple
 * sweep counts the admissible (speed node, control) pairs times all SoC and
 * time nodes.  dp_instance_info.evaluations is the dense count (every node
 * times every control) that the throughput figures use.  Synchronises on
 * `stream`. */
int dp_executed_evaluations(dp_plan *p, int64_t *counts, void *stream);

/* Synchronises on `stream` and reads the plan's device error word, which
 * kernels set when they meet a condition the host checks could not exclude
 * (a SoC cell offset outside the int8 field of the sweep's records, a
 * persistent sweep that gave up waiting, a negative device terminal_V).
 * DP_OK if it is clear; else DP_EDEVICE with the condition named in
 * dp_last_error(), and the word is cleared.  Results of the solves enqueued
 * before such an error are not to be used. */
int dp_device_check(dp_plan *p, void *stream);

/* With DP_TIMING: total device milliseconds and launch count of the state
 * sweep kernel over every dp_solve / dp_stage since the previous call
 * (synchronises on the recorded events, then starts a new count). */
int dp_sweep_time(dp_plan *p, double *ms, int32_t *launches);

void dp_destroy(dp_plan *p);
const char *dp_status_string(int code);
int dp_last_error(char *buf, size_t n);

#ifdef __cplusplus
}
#endif
#endif
