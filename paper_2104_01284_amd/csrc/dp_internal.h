// Internal declarations of the ecodp library (host launch wrappers).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/ecodp.h"
#include "dp_model.h"

namespace ecodp {

// Every instance's terminal slab (grid y = instance) and root step in one
// launch each; per-instance byte offsets of J_N and J_1 from J.
int launch_terminal_jobs(const DevInst *insts, int n_inst, long max_slab, void *J, const long long *jN_off,
                         int *err, hipStream_t s);
int launch_terminal_shift(const float *src, long nvs, int n_src, double h_src, double t_shift, int n_dst, double h_dst,
                          double Jinf, float *dst, hipStream_t s);
int launch_stage_table(const DevInst &P, int k, StageEntry *st, BatEntry *bat, unsigned long long *count,
                       hipStream_t s);
int launch_sweep(const DevInst &P, int k, const float *Jn, float *Jk, int16_t *pik, const StageEntry *st,
                 const BatEntry *bat, const TLEntry *tl, hipStream_t s);
int launch_root_jobs(const DevInst *insts, int n_inst, const void *J, const long long *j1_off, float *V0, int16_t *u0,
                     hipStream_t s);

// Grouped sweep geometry: floats per staged plane row (time nodes plus at
// least one padding column, rounded up to 32 so that the rows of a small grid
// do not waste LDS), staged SoC rows
// of a tile of JT rows whose successor cells move by at most H, and threads
// per workgroup (a wave covers 63 time nodes plus the neighbour of the last;
// a tile of more than 8 rows runs on JT / 8 such groups of waves).
inline int sweep_pitch(int n_t) { return ((n_t + 1 + 31) / 32) * 32; }
inline int sweep_rows(int JT, int H) { return JT + 2 * H + 1; }
inline int sweep_threads(int JT, int n_t) { return (JT > 8 ? JT / 8 : 1) * 64 * ((n_t + 62) / 63); }

// Grouped sweep over a table of (instance, stage) jobs.
int launch_stage_jobs(const StageBase &B, int njobs, int max_nv, long max_records, hipStream_t s);
size_t lds_sweep_bytes(int JT, int H, int n_t);
size_t lds_sweep_bytes_p(int JT, int H, int pitch, int threads);
size_t lds_job_index_bytes(int njobs);
int sweep_vgprs(int JT, int pitch);
int launch_sweep_jobs(int JT, int pitch, int threads, const StageBase &B, int njobs, const int *item_begin,
                      int total, int *queue, int grid, size_t lds, hipStream_t s);
int launch_combine_jobs(const StageBase &B, int njobs, long max_nodes, hipStream_t s);
// The persistent multi-instance sweep of one kernel class (JT rows, LDS pitch).
int launch_sweep_persist(int JT, int pitch, int threads, const StageBase &B, const DevInst *insts,
                         const PersistQueues &Q, int grid, size_t lds, hipStream_t s);
// Resident workgroups per CU of that kernel (0 if unknown).
int persist_blocks_per_cu(int JT, int pitch, int threads, size_t lds);
int launch_fill_i32(int *p, long n, int v, hipStream_t s);

// Every instance's rollout in one launch (one wave each); offsets per instance.
int launch_rollout_jobs(const DevInst *insts, int n_inst, const void *pi, const long long *pi_off,
                        const long long *traj_off, const int16_t *u0, double *traj, int32_t *status, hipStream_t s);
int launch_fill_f64(double *p, long n, double v, hipStream_t s);
int launch_adjoint_root(const DevInst &P, const float *J1, const int16_t *u0, double *rho1, double *gacc,
                        double *gstage, hipStream_t s);
// The stage table of the adjoint (per speed node and control) and one stage
// of the occupancy sweep; rho is zeroed as it is read.
size_t adjoint_table_bytes(const DevInst &P);
int launch_adjoint_table(const DevInst &P, int k, void *tab, hipStream_t s);
int launch_adjoint_stage(const DevInst &P, int k, const float *Jn, const int16_t *pik, const TLEntry *tl,
                         const void *tab, double *rho, double *rho_next, double *gacc, double *gstage,
                         double *gspat_L, bool wide, hipStream_t s);
// dspat[3 L + (0, 1, 2)] = dV/d(offset, red, cycle) of signal L from the
// adjoint_grade_slots() slot pairs per signal in gspat.
int launch_adjoint_spat(int n_lights, const double *gspat, const double *grad, double *dspat, hipStream_t s);
int launch_adjoint_grade(const DevInst &P, const double *gstage, const double *grad, double *dgrade, hipStream_t s);
size_t adjoint_grade_slots();
// gpart: the adjoint kernels' per-workgroup partial gradient sums (1024 x 5
// doubles, zeroed before the first stage); grad += their sum.
int launch_adjoint_reduce(const double *gpart, double *grad, hipStream_t s);
int launch_adjoint_terminal(const DevInst &P, const float *JN, const double *rho, double *gacc, hipStream_t s);

// ---- plans kept by a closed loop (dp_loop.hip) ----
// Records the error message dp_last_error reports; returns code.
int api_fail(int code, const char *fmt, ...);
// A one-instance plan of a horizon window: built like dp_build_problem, but
// every stage builds its own tables (the window moves along a route) and the
// SoC-shift bound is at least H_min (the route's).  The description must carry
// a signal at every stage 1..N-1 (placeholders until plan_set_window).
int build_window_plan(const dp_problem_desc &d, int H_min, const dp_options *opt, int device, dp_plan **out);
// Moves a window plan to another window of its route in place: grade [N],
// speed limits [N+1], per stage 1..N-1 a signal (cycle, red, offset, yellow;
// red = yellow = 0 for a stage without one), clock and initial state, uploaded through the
// plan's pinned staging on stream s.  Recorded graphs pick it up on replay.
int plan_set_window(dp_plan *p, const double *grade, const double *vmax, const double *cycle, const double *red,
                    const double *offset, const double *yellow, double t0_abs, double v0, double soc0, hipStream_t s);
// The plan's own device copy of its terminal table (DP_TERMINAL_DEVICE), or NULL.
float *plan_terminal(dp_plan *p);

}  // namespace ecodp
