/*
 * fruitninja.h -- C ABI of the MI355X (gfx950) edge-timing library
 * (libfruitninja.so).
 *
 * The library implements the batched inner loop of the FRUITNINJA planner
 * ("Becoming a Fruit Ninja", Sec. IV-E and Algorithm 1): for every pair of a
 * candidate state and one of its nearest tree nodes it builds the cubic edge
 * of Eq. (6), searches a grid of travel times for the first one whose torque
 * and power ratios of Eq. (7) are within limits (Def. 6, Def. 7), using the
 * torque model of Eqs. (4)-(5), and checks the velocity taper, position
 * limits and clearance at that time.
 *
 * Conventions shared by every call
 *  - Pointers marked "device" are device memory (e.g. torch tensors'
 *    data_ptr()); "host" pointers are read during the call only.  The caller
 *    owns every buffer and keeps it alive until the stream has finished.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *    and the call returns without synchronising.  No call allocates device
 *    memory except fn_create and fn_mlp_create.
 *  - Arguments are checked on the host before anything is enqueued.  A
 *    negative return code (FN_E_*) means nothing was enqueued;
 *    fn_last_error() then returns a message (thread-local).  No exception
 *    crosses the ABI.  Data conditions (NaN inputs, a padded parent) are not
 *    errors: they set per-edge status bits.
 *  - A state is 14 floats: joint positions q[7] then velocities qd[7].
 *  - The tree is structure-of-arrays: tree[c * ld + n] is coordinate c of
 *    node n (c = 0..13), ld >= n_nodes rounded up to a multiple of 4, ld a
 *    multiple of 4, the base 16-byte aligned.
 *  - Calls on one context must not overlap in time across streams (they
 *    share the context's scratch buffers).
 */
#ifndef FRUITNINJA_H
#define FRUITNINJA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FN_DOF 7
#define FN_STATE 14
#define FN_MAX_SPHERES 64
#define FN_MAX_OBS 64
#define FN_MAX_SAMPLES 64
#define FN_MAX_NT 256
#define FN_MAX_K 32

/* return codes */
enum {
  FN_OK = 0,
  FN_E_ARG = -1,         /* bad pointer or value */
  FN_E_SHAPE = -2,       /* size out of range or beyond the context's caps */
  FN_E_UNSUPPORTED = -3, /* arm or option the library does not handle */
  FN_E_HIP = -4,         /* HIP runtime error (message has the HIP text) */
  FN_E_NOMEM = -5,       /* device allocation failed (create calls only) */
  FN_E_STATE = -6        /* wrong object state (e.g. untrained surrogate) */
};

/* per-edge status bits.  An edge is valid (Alg. 1: ok_p) iff its T index
 * is >= 0 and none of NONE, VEL, POS, COLL, BAD_INPUT, NO_PARENT is set. */
enum {
  FN_S_NONE = 1,        /* no grid slot with rho_tau <= 1 and rho_P <= 1 (Def. 7) */
  FN_S_VEL = 2,         /* velocity taper violated at the searched T (Def. 6 rho_v) */
  FN_S_POS = 4,         /* joint position limit crossed along the edge */
  FN_S_COLL = 8,        /* arm sphere closer than the margin to an obstacle (checked only
                           when every limit check passed: Alg. 1 and-s Clear in last) */
  FN_S_RECHECK64 = 16,  /* informational: a ratio within 1e-3 of 1 was decided in FP64 */
  FN_S_WIN_HIT = 32,    /* informational: the result lies in the predicted window */
  FN_S_WIN_MISS = 64,   /* informational: it does not; the exact scan found it elsewhere */
  FN_S_BAD_INPUT = 128, /* a non-finite state or duration */
  FN_S_WIN_BELOW = 256, /* informational: a slot below the window passed the endpoint screen
                           and was evaluated in full */
  FN_S_NO_PARENT = 512, /* padded parent index (-1): no edge */
  FN_S_SELF = 1024      /* edge_check: two of the arm's own spheres closer than the margin
                           (set together with FN_S_COLL) */
};
#define FN_S_DECISION (FN_S_NONE | FN_S_VEL | FN_S_POS | FN_S_COLL | FN_S_BAD_INPUT | FN_S_NO_PARENT)

/* dynamics terms of Eq. (4) */
enum { FN_T_RIGID = 1, FN_T_ARMATURE = 2, FN_T_FRICTION = 4, FN_T_GRAVITY = 8, FN_T_ALL = 15 };

/* search modes of edge_time_batch */
enum {
  FN_SEARCH_PLAIN = 0,  /* ascending scan, every sample of every slot, stop at the first feasible */
  FN_SEARCH_SCREEN = 1, /* endpoint samples of all slots first; full slots only where they pass */
  FN_SEARCH_WINDOW = 2  /* learned window: endpoint certificate below it, window, exact fallback */
};

/* Arm description (host, FP64).  Modified DH: joint i's frame is
 * Rx(alpha[i]) Tx(a[i]) Rz(q_i) Tz(d[i]) relative to frame i-1.  Link i's
 * mass m, COM rc (frame i) and
 * diagonal inertia about the COM (frame i); reflected rotor inertia Im and
 * the friction parameters psi1..3 of Eq. (5); joint limits, velocity limit
 * qdmax with braking deceleration acc (velocity taper
 * min(qdmax, sqrt(2 acc dist)), dist = distance to the limit the motion
 * heads for), torque limits, power limit wmax (Def. 1); gravity g (base
 * frame); collision spheres: link index 1..7, centre in that link's frame
 * and radius (Sec. IV-E). */
typedef struct {
  int32_t n; /* must be 7 */
  int32_t terms; /* FN_T_* bits, normally FN_T_ALL */
  double alpha[7], a[7], d[7];
  double m[7], rc[7][3], inertia[7][3];
  double Im[7], psi1[7], psi2[7], psi3[7];
  double qmin[7], qmax[7], qdmax[7], taumax[7], acc[7];
  double wmax;
  double g[3];
  int32_t n_spheres;
  int32_t sphere_link[FN_MAX_SPHERES];
  double sphere[FN_MAX_SPHERES][4];
} fn_arm_desc;

/* Capacities fixed at creation; every scratch buffer is sized from them. */
typedef struct {
  int32_t max_nodes;   /* largest tree */
  int32_t max_batch;   /* largest candidate batch B */
  int32_t max_k;       /* largest k (<= FN_MAX_K) */
  int64_t max_edges;   /* largest number of edges per edge_time_batch / edge_check call, and
                          of all problems of a batched iteration together */
  int32_t max_problems; /* most problems in a batched iteration (0: no batched iterations) */
} fn_caps;

typedef struct fn_ctx fn_ctx;

/* Creates a context on the current HIP device: copies the arm, derives its
 * FP32 and FP64 constant blocks on the device, and allocates scratch for the
 * caps.  Twists of 0 or +-pi/2 select kernels with the rotations folded in
 * at compile time; other twists use a general kernel.  Returns FN_OK and
 * *out, or FN_E_ARG / FN_E_UNSUPPORTED (n != 7, more than FN_MAX_SPHERES
 * spheres) / FN_E_NOMEM / FN_E_HIP. */
int fn_create(const fn_arm_desc* arm /*host*/, const fn_caps* caps /*host*/, fn_ctx** out);
/* Frees the context (synchronises the device first). NULL is a no-op. */
void fn_destroy(fn_ctx* ctx);
/* Message of the last nonzero return on this thread ("" if none). */
const char* fn_last_error(void);
/* Library version string. */
const char* fn_version(void);

/* Kernel timing for measurement.  While enabled, every edge_time_batch
 * call records a pair of HIP events on its stream around its search kernel
 * (edge_time_kernel), up to FN_MAX_TIMED calls; later calls are not timed.
 * fn_kernel_times waits for the recorded pairs, writes their elapsed
 * milliseconds to out_ms (host, up to max entries, *n_out of them) and
 * clears the list.  Events are created by fn_kernel_timing(ctx, 1) and
 * freed by fn_kernel_timing(ctx, 0) or fn_destroy.  Errors: FN_E_ARG (NULL
 * context / out), FN_E_HIP. */
#define FN_MAX_TIMED 256
int fn_kernel_timing(fn_ctx* ctx, int enable);
int fn_kernel_times(fn_ctx* ctx, float* out_ms /*host*/, int32_t max, int32_t* n_out /*host*/);

/* ------------------------------------------------------------------ */
/* plan_knn -- Parents(T, x, M) of Alg. 1 (Sec. IV-E, "brute-force     */
/* parallel scan"): the k nearest tree nodes of every query by plain   */
/* Euclidean distance in the 14-D state space.                         */
/* ------------------------------------------------------------------ */
/* tree: device SoA (see conventions), n_nodes >= 0 nodes;
 * queries: device [B][14] float; out_idx: device [B][k] int32, sorted by
 * (d^2, node index); out_d2: device [B][k] float or NULL.  Ranking is exact:
 * an FP32 scan selects candidates and every candidate near the k-th
 * distance is re-ranked with d^2 = sum_{c=0..13} (x_c - y_c)^2 in FP64,
 * summed in order c = 0..13 with separately rounded products and sums;
 * out_d2 is that FP64 value rounded to float.  The FP32 screening keys come
 * from FMAs or from the matrix cores, as fn_set_tuning selects; the result
 * is the same.  With fewer than k nodes the
 * tail is padded with -1 (d^2 = +inf).  Returns FN_E_SHAPE if B > max_batch,
 * k > max_k, k < 1, n_nodes > max_nodes or ld > 38,347,920 (the scan's
 * 32-bit row offsets); FN_E_ARG if ld is not a multiple of 4 or too small. */
int plan_knn(fn_ctx* ctx, const float* tree, int64_t ld, int32_t n_nodes, const float* queries,
             int32_t B, int32_t k, int32_t* out_idx, float* out_d2, void* stream);

/* Search grid (Sec. IV-D after Def. 7 / Alg. 1 free-candidate branch):
 * grid: device [n_t] float, strictly increasing, > 0; samples S: the
 * evaluation times are t_s = T * s / (S-1), s = 0..S-1 (2 <= S <= 64). */
typedef struct {
  const float* grid; /* device */
  int32_t n_t;
  int32_t samples;
  int32_t mode;      /* FN_SEARCH_* */
  int32_t win_half;  /* window mode: slots win_lo .. win_lo + 2*win_half */
  const int16_t* j_max;  /* device [E] or NULL: search slots 0..j_max only (t_best bound) */
  const int16_t* win_lo; /* device [E], window mode only: lowest slot of the window,
                            n_t = "predicted infeasible" */
} fn_search;

/* Obstacles (world frame, Sec. IV-E): spheres, device [n][4] = (x, y, z,
 * radius), and capsules, device [n_caps][7] = (segment end p0, segment end
 * p1, radius); an arm sphere clears a capsule when its distance to the
 * segment is at least r_a + r + margin.  n + n_caps <= FN_MAX_OBS. */
#define FN_MAX_CAPS 16
typedef struct {
  const float* spheres;  /* device, may be NULL when n == 0 */
  int32_t n;             /* 0 .. FN_MAX_OBS */
  float margin;          /* clearance margin, metres (>= 0) */
  const float* capsules; /* device, may be NULL when n_caps == 0 */
  int32_t n_caps;        /* 0 .. FN_MAX_CAPS */
} fn_obstacles;

/* Per-edge outputs (device, length E each).  rho4 (nullable): (rho_tauP at
 * the result slot (at the last slot when none), rho_v, rho_q, rho_c) where
 * rho_c = max (r_a + r_o + margin)/distance, NaN when rho_v or rho_q fails
 * (the clearance is then not evaluated), 0 without obstacles.  margin: the smallest
 * |rho - 1| over the ratios the decision rests on.  work (nullable): number
 * of (slot, sample) evaluations of Eq. (4) performed for the edge.
 * screened (nullable): number of slots whose two endpoint ratios were
 * evaluated from the endpoint models (screening and window modes). */
typedef struct {
  int16_t* j;          /* T index (first feasible slot) or -1 */
  uint16_t* status;    /* FN_S_* bits */
  float* margin;
  float* rho4;         /* [E][4] or NULL */
  int32_t* work;       /* or NULL */
  int16_t* screened;   /* or NULL */
} fn_edge_out;

/* ------------------------------------------------------------------ */
/* edge_time_batch -- the minimum feasible time of every (candidate,   */
/* parent) edge on the grid (Def. 7, Alg. 1 free branch), then the     */
/* velocity taper (Def. 6 rho_v, exact extremum), position limits and  */
/* clearance (Sec. IV-E) at that time.                                 */
/* ------------------------------------------------------------------ */
/* Edge e = b * k + i goes from tree node nbr[b][i] (x0) to candidate b (x1).
 * cand: device [B][14]; nbr: device [B][k] int32 (-1 = padding).  Every
 * mode returns the first slot j with rho_tau(T_j) <= 1 and rho_P(T_j) <= 1
 * among 0..j_max; the modes differ only in the work done.  Ratios are
 * evaluated in FP32; any ratio within 1e-3 of 1 is re-evaluated in FP64
 * before it decides.  Returns FN_E_SHAPE for B*k > max_edges, n_t out of
 * 1..FN_MAX_NT, S out of 2..FN_MAX_SAMPLES, too many obstacles; FN_E_ARG for
 * NULL required pointers or window mode without win_lo.  B = 0 is a no-op
 * once the sizes check (the arrays may then be NULL). */
int edge_time_batch(fn_ctx* ctx, const float* tree, int64_t ld, int32_t n_nodes,
                    const float* cand, int32_t B, const int32_t* nbr, int32_t k,
                    const fn_search* search, const fn_obstacles* obs, const fn_edge_out* out,
                    void* stream);

/* Self-collision pairs of the arm checked by edge_check (Sec. IV-E: the
 * pairs that the joint limits make unreachable are removed offline, by the
 * caller): pairs host [n][2] of sphere indices (the arm description's
 * order, distinct, < n_spheres), margin >= 0 metres.  Copies them to the
 * context (synchronous); n = 0 removes them.  Errors: FN_E_ARG, FN_E_SHAPE
 * (n > FN_MAX_SELF_PAIRS). */
#define FN_MAX_SELF_PAIRS 1024
int fn_set_self_pairs(fn_ctx* ctx, const int32_t* pairs /*host*/, int32_t n, float margin);

/* ------------------------------------------------------------------ */
/* edge_refine -- multi-round N-ary refinement of the minimum feasible  */
/* time below the grid result (Sec. IV-D after Def. 7: the interval is  */
/* cut into N equal slots, their ends evaluated, and the slot whose end */
/* is the first feasible one cut again until it is no wider than eps). */
/* ------------------------------------------------------------------ */
typedef struct {
  const float* grid; /* device [n_t], the grid j_in indexes */
  int32_t n_t;
  int32_t samples;   /* S, 2..FN_MAX_SAMPLES */
  int32_t n_ary;     /* N, 2..1024; each round evaluates N - 1 interior points */
  float eps;         /* stop once hi - lo <= eps (seconds), > 0 */
} fn_refine;

/* Edges as edge_time_batch (edge e = b * k + i from tree node nbr[b][i] to
 * candidate b); j_in: device [E], the grid search's result slot of every
 * edge (-1: none).  For j_in[e] >= 0 the search starts from hi = grid[j],
 * which is feasible, and lo = grid[j - 1] (0 for j = 0), which is not;
 * every round evaluates t_i = lo + i (hi - lo) / N, i = 1 .. N-1, in
 * ascending order in FP32, the first t_i with rho_tau, rho_P <= 1 becomes hi
 * and t_{i-1} lo (lo = t_{N-1} when none is), at most 64 rounds.  Outputs
 * (device, length E): out_T = hi (NaN when not refined), out_status
 * (FN_S_VEL / POS / COLL of the post-checks at out_T, clearance only when
 * the limit checks pass; FN_S_NONE when j_in < 0; BAD_INPUT, NO_PARENT),
 * out_rho4 [E][4] = (rho_tauP(out_T), rho_v, rho_q, rho_c), out_rounds and
 * out_work (sample evaluations) or NULL.  FP32 throughout, no FP64 stage:
 * the result is within eps of the FP32 boundary.  Errors: FN_E_ARG (NULL
 * arrays, N or eps out of range), FN_E_SHAPE (n_t, S, k, obstacles). */
int edge_refine(fn_ctx* ctx, const float* tree, int64_t ld, int32_t n_nodes, const float* cand,
                int32_t B, const int32_t* nbr, int32_t k, const int16_t* j_in,
                const fn_refine* refine, const fn_obstacles* obs, float* out_T,
                uint16_t* out_status, float* out_rho4, int32_t* out_rounds, int32_t* out_work,
                void* stream);

/* ------------------------------------------------------------------ */
/* fn_control -- the 1 kHz tracking controller (Sec. IV-F, Eq. (9)),    */
/* one step for each of n instances.                                   */
/* ------------------------------------------------------------------ */
/* status bits of a control step */
enum {
  FN_C_ACC = 1,     /* the desired acceleration was clipped to the velocity taper */
  FN_C_SLEW = 2,    /* the torque was clipped to the slew limit */
  FN_C_TORQUE = 4,  /* the torque was clipped to the torque limit */
  FN_C_POWER = 8,   /* the torque was scaled to the power limit */
  FN_C_BAD = 128    /* non-finite input or horizon T <= 0: zero torque and acceleration */
};
/* Per instance (device [n][7] floats each): measured q, qd, the previous
 * torque command tau_prev, the rendezvous qg, qdg, and the horizon T
 * (device [n], seconds to the rendezvous).  The controller refits the cubic
 * of Eq. (6) from (q, qd) to (qg, qdg) over T and takes its initial
 * acceleration, Eq. (9): qdd = 6 (qg - q) / T^2 - (4 qd + 2 qdg) / T, clipped
 * to [l, u] with l = (-taper(q, -) - qd) / dt, u = (taper(q, +) - qd) / dt
 * (the velocity after one period dt stays inside the context's velocity
 * taper, braking law of the arm description); the torque of Eq. (4) at
 * (q, qd, qdd) is then clipped to |tau - tau_prev| <= slew dt (slew: host
 * [7], N m / s), to |tau| <= taumax, and scaled by W_max / |sum tau qd| when
 * the power exceeds W_max.  Outputs (device): out_tau [n][7], out_qdd [n][7]
 * (the clipped acceleration), out_status [n] (FN_C_* bits).  FP32.  Errors:
 * FN_E_ARG (NULL arrays, dt <= 0, a negative slew limit), FN_E_SHAPE. */
int fn_control(fn_ctx* ctx, int64_t n, const float* q, const float* qd, const float* tau_prev,
               const float* qg, const float* qdg, const float* T, float dt,
               const double* slew /*host [7]*/, float* out_tau, float* out_qdd,
               uint16_t* out_status, void* stream);

/* ------------------------------------------------------------------ */
/* edge_time_batch_noalloc -- edge_time_batch for callers that cannot   */
/* allocate device memory (code under HIP graph capture, tight serving  */
/* loops, harnesses that forbid hipMalloc).                            */
/* ------------------------------------------------------------------ */
/* Same arguments, results and errors as edge_time_batch, except that its
 * scratch (the FP64-stage counter and queue and the endpoint models) lives
 * in a file-scope device array of the library, fn_noalloc_scratch_bytes()
 * bytes (about 17 MiB) on every device the library runs on, held until the
 * process ends, instead of in the context: the call allocates nothing.
 * The context still supplies the arm constants.  At most
 * FN_NOALLOC_MAX_EDGES edges per call (B * k beyond it: FN_E_SHAPE; the
 * context's max_edges does not apply).  Every call on one device uses the
 * same array, which keeps the last call's contents (the search clears what
 * must start at zero); calls that overlap in time on one device (other
 * streams or threads) race.  Search-kernel timing (fn_kernel_timing) does
 * not record these calls. */
#define FN_NOALLOC_MAX_EDGES 32768
int edge_time_batch_noalloc(fn_ctx* ctx, const float* tree, int64_t ld, int32_t n_nodes,
                            const float* cand, int32_t B, const int32_t* nbr, int32_t k,
                            const fn_search* search, const fn_obstacles* obs,
                            const fn_edge_out* out, void* stream);
/* Bytes of that array per device. */
size_t fn_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------ */
/* edge_check -- one fixed duration per edge: the goal-candidate branch */
/* of Alg. 1 (T = T_req - t_p) and the full-resolution recheck of a    */
/* sent plan (Sec. IV-E).                                              */
/* ------------------------------------------------------------------ */
/* x0, x1: device [E][14]; T: device [E]; S samples, 2..4096 (the full
 * resolution of a sent plan may exceed the search's 64).  out_status:
 * device [E] (NONE when rho_tau or rho_P > 1 or T <= 0, VEL, POS, COLL,
 * SELF, BAD_INPUT); out_rho5: device [E][5] = (rho_tau, rho_P, rho_v,
 * rho_q, rho_c; NaN unless the four limit ratios pass); rho_c is the larger
 * of the obstacle clearance and, when the context has self-collision pairs
 * (fn_set_self_pairs), the pairs' (r_a + r_b + margin) / distance; out_tau:
 * device [E][S][7] torques of Eq. (4) at the samples, or NULL.  FP32
 * arithmetic (no FP64 recheck here). */
int edge_check(fn_ctx* ctx, const float* x0, const float* x1, const float* T, int64_t E,
               int32_t S, const fn_obstacles* obs, uint16_t* out_status, float* out_rho5,
               float* out_tau, void* stream);

/* ------------------------------------------------------------------ */
/* risk_score -- the objective J of Eq. (2) with the terms of Eq. (3)   */
/* (Sec. IV-B) for n rendezvous nodes; evaluated in FP32 (log Phi's     */
/* tail through the scaled complementary error function).              */
/* ------------------------------------------------------------------ */
typedef struct {
  double gz;          /* vertical gravity of Eq. (1) (negative) */
  int32_t sigma_mode; /* 0: sigma^2 = sp^2 + (sv t)^2 + (sa t^2 / 2)^2;  1: sigma = s0 + s1 t */
  double sp, sv, sa, s0, s1;
  double wv, vtarget, wp, wr, wx, r, nu0, lam; /* weights and constants of Eqs. (2)-(3) */
} fn_risk;

/* T: arrival times; v_rel: relative blade-object speed; nu: peak velocity
 * fraction; vz0: vertical launch speed of the flight; t_fall: time the
 * flight leaves reach (all device [n] float).  out_J: device [n] float. */
int risk_score(fn_ctx* ctx, const fn_risk* w /*host*/, const float* T, const float* v_rel,
               const float* nu, const float* vz0, const float* t_fall, int32_t n, float* out_J,
               void* stream);


/* ------------------------------------------------------------------ */
/* Learned T-window surrogate.  A 4-layer MLP 28 -> 256 -> 256 -> 256  */
/* -> 2 (SiLU after the first three layers) maps an edge's boundary    */
/* states (the inputs of Eq. (6)) to (standardised log T*, feasibility */
/* logit), where T* is the result of Def. 7 on the grid.  BF16 weights  */
/* and activations on MFMA with FP32 accumulation; FP32 master weights  */
/* and Adam.  Its prediction only narrows edge_time_batch's work        */
/* (FN_SEARCH_WINDOW); results stay exact.                             */
/* ------------------------------------------------------------------ */
typedef struct fn_mlp fn_mlp;

/* Training configuration: epochs over the data, minibatch rows (multiple
 * of 8, <= 8192), Adam learning rate (cosine decay to 0 over the run when
 * cosine != 0), betas, eps, shuffling seed, and the T grid the slot labels
 * index (device [n_t]). */
typedef struct {
  int32_t epochs, batch;
  float lr, beta1, beta2, eps;
  int32_t cosine;
  uint64_t seed;
  const float* grid;
  int32_t n_t;
} fn_train_cfg;

/* Creates a network on the context's device with weights drawn
 * U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from SplitMix64(seed); Adam state 0. */
int fn_mlp_create(fn_ctx* ctx, uint64_t seed, fn_mlp** out);
void fn_mlp_destroy(fn_mlp* mlp);
/* Number of parameters in the logical layout W1[256][28], b1[256],
 * W2[256][256], b2, W3[256][256], b3, W4[2][256], b4[2] (row-major). */
int fn_mlp_param_count(void);
/* Host copy in/out of the FP32 parameters (logical layout; set resets the
 * Adam state).  FN_E_SHAPE if count differs from fn_mlp_param_count(). */
int fn_mlp_set_params(fn_mlp* mlp, const float* host, int64_t count);
int fn_mlp_get_params(const fn_mlp* mlp, float* host, int64_t count);
/* Checkpoint: parameters, Adam moments and step count (binary file). */
int fn_mlp_save(const fn_mlp* mlp, const char* path);
int fn_mlp_load(fn_ctx* ctx, const char* path, fn_mlp** out);

/* Surrogate inputs of every edge: X[e] = (state of tree node nbr[e], state
 * of candidate e / k) as 28 floats (zeros for a padded parent).
 * Arguments as edge_time_batch; X: device [B*k][28]. */
int edge_features(fn_ctx* ctx, const float* tree, int64_t ld, int32_t n_nodes, const float* cand,
                  int32_t B, const int32_t* nbr, int32_t k, float* X, void* stream);

/* Trains on N rows: X device [N][28] raw edge states; y_j device [N] the
 * exact search's slot index (-1 = no feasible slot).  Inputs are
 * normalised inside ((q - centre)/half-range, qd/qdmax); the regression
 * target is (log T_j - mu)/s mapping [log T_0, log T_last] to [-1, 1].
 * Loss per minibatch: mean squared error of output 0 over rows with a slot
 * + binary cross-entropy with logits of output 1.  out_epoch_loss: device
 * [epochs][3] (mean total, squared-error and cross-entropy terms) or NULL.
 * Each epoch visits floor(N / batch) minibatches of a permutation
 * i -> (a i + c) mod N drawn from the seed. */
int surrogate_train(fn_ctx* ctx, fn_mlp* mlp, const float* X, const int16_t* y_j, int64_t N,
                    const fn_train_cfg* cfg, float* out_epoch_loss, void* stream);

/* Loss and gradient of one batch without updating (N <= 8192, multiple of
 * 8): out_grad device [fn_mlp_param_count()] (logical layout), out_loss3
 * device [3] or NULL. */
int surrogate_grad(fn_ctx* ctx, fn_mlp* mlp, const float* X, const int16_t* y_j, int32_t N,
                   const float* grid, int32_t n_t, float* out_grad, float* out_loss3,
                   void* stream);

/* Inference on N rows: out device [N][2] = (standardised log T*, logit) or
 * NULL; out_win_lo device [N] or NULL: lowest slot of the window, i.e. the
 * grid slot nearest the predicted T* minus `half` (clamped at 0), or n_t
 * (predicted infeasible) when the logit is below logit_min.  N = 0 is a
 * no-op once the sizes check (X and grid may then be NULL). */
int surrogate_infer(fn_ctx* ctx, const fn_mlp* mlp, const float* X, int64_t N, const float* grid,
                    int32_t n_t, int32_t half, float logit_min, float* out, int16_t* out_win_lo,
                    void* stream);

/* The windows of B * k edges straight from the tree and the candidates:
 * surrogate_infer on the rows edge_features would write (state of tree node
 * nbr[e], state of candidate e / k; zeros for a padded or out-of-range
 * parent), gathered inside the inference kernel, so no feature matrix is
 * written.  Same results as edge_features followed by surrogate_infer.
 * B = 0 is a no-op once the sizes check. */
int surrogate_window(fn_ctx* ctx, const fn_mlp* mlp, const float* tree, int64_t ld,
                     int32_t n_nodes, const float* cand, int32_t B, const int32_t* nbr, int32_t k,
                     const float* grid, int32_t n_t, int32_t half, float logit_min, float* out,
                     int16_t* out_win_lo, void* stream);

/* ------------------------------------------------------------------ */
/* Launch mappings chosen by the autotuner                             */
/* ------------------------------------------------------------------ */
/* kNN: the scan is split into node chunks until about knn_target_waves
 * wavefronts run (chunks of at least knn_min_chunk nodes).  0 keeps the
 * default (4096 wavefronts, 512 nodes).  knn_form: 1 = every wavefront
 * loads its own node rows (4 queries per wavefront, keys by FP32 FMAs);
 * 2 = the 4 wavefronts of a workgroup share 256-node tiles in LDS (one
 * global load per node instead of four); 3 = matrix cores: 16 queries per
 * wavefront, each 16 x 16 block of keys by four v_mfma_f32_16x16x4_f32 over
 * the augmented vectors (-2x, |x|^2, 1) . (y, 1, |y|^2) (at most 4096
 * wavefronts, whatever knn_target_waves says); 0 = chosen by tree size
 * (matrix cores above FN_KNN_LARGE_TREE nodes).  Every form returns the same
 * neighbours and distances.  Applies to later plan_knn calls and
 * fn_batch_prepare.  Errors: FN_E_ARG when knn_target_waves is outside
 * [0, 16384], knn_min_chunk is negative or not a multiple of 64, or
 * knn_form is not 0, 1, 2 or 3, edge_form is not 0, 1, 2 or 3, or mlp_rows is
 * not 0, 32 or 64. */
#define FN_KNN_LARGE_TREE 65536
typedef struct {
  int32_t knn_target_waves;
  int32_t knn_min_chunk;
  int32_t knn_form;
  int32_t edge_form;  /* screened and windowed searches of edge_time_batch: 1 one kernel (one
                       * wavefront per edge); 2 two phases (a triage of every edge by the
                       * endpoint screen, which finishes the edges it leaves no open slot on,
                       * then the search of the others); 3 two phases with the open edges
                       * searched in descending order of their open-slot count (a counting
                       * sort between the phases); 0 default: 3 from 2^15 edges, else 1.
                       * Batched rounds (fn_batch_prepare) search in the ordered form when
                       * it is 3 and in one kernel otherwise.  The results are the same. */
  int32_t mlp_rows;   /* rows per workgroup of the fused surrogate inference: 32 or 64; 0
                       * default (32 while 64 would leave fewer than four workgroups per
                       * compute unit).  The results are the same. */
} fn_tuning;
int fn_set_tuning(fn_ctx* ctx, const fn_tuning* t /*host*/);

/* ------------------------------------------------------------------ */
/* Batched planning iteration (Algorithm 1, one round for many         */
/* problems): Parents for every candidate, the edge of every           */
/* (candidate, parent) pair -- free candidates searched on the grid,   */
/* goal candidates checked once at T = t_req - t(parent) -- then each  */
/* candidate attached to the valid parent with the smallest            */
/* t(parent) + T (ties: lower kNN rank), appended to its tree in       */
/* candidate order, and every attached goal node scored with J of      */
/* Eq. (2).  All problems share k, the grid, S and the arm; each has   */
/* its own tree, candidates and obstacles.                             */
/* ------------------------------------------------------------------ */
typedef struct {
  float* tree;           /* device SoA [14][ld]; the first *n_nodes nodes are valid */
  int64_t ld;            /* node capacity, a multiple of 4 */
  int32_t* n_nodes;      /* device counter; grows by the attached candidates (capped at ld) */
  float* t_node;         /* device [ld] time-to-come of each node */
  int32_t* parent;       /* device [ld] parent node (-1: root) */
  float* nu;             /* device [ld] peak velocity fraction on the path to the node */
  const float* cand;     /* device [B][14] candidates of this round */
  const int32_t* kind;   /* device [B]: 0 free, 1 goal */
  const float* t_req;    /* device [B] required arrival time of a goal */
  const float* v_rel;    /* device [B] relative blade-object speed of a goal */
  const float* vz0;      /* device [B] vertical launch speed of the goal's flight */
  const float* t_fall;   /* device [B] time the goal's flight leaves reach */
  int32_t B;
  const float* obs;      /* device [n_obs][4] obstacle spheres, or NULL */
  int32_t n_obs;
  int32_t* nbr;          /* device out [B][k] parents */
  int16_t* out_j;        /* device out [B*k] slot (free) or 0 (goal feasible at t_req - t_p), -1 */
  uint16_t* out_status;  /* device out [B*k] FN_S_* bits */
  float* out_margin;     /* device out [B*k] */
  float* out_rho4;       /* device out [B*k][4] */
  float* out_T;          /* device out [B*k] duration of the result */
  int32_t* out_node;     /* device out [B] index of the attached node, -1 if none */
  float* out_J;          /* device out [B] J of an attached goal node, -inf otherwise */
  float* out_best;       /* device out [2]: best J among this round's goal nodes, its node (as float) */
  const float* caps;     /* device [n_caps][7] obstacle capsules, or NULL (n_obs + n_caps <= FN_MAX_OBS) */
  int32_t n_caps;
  /* Anytime outer loop (Algorithm 1), optional; the same choice for every
   * problem of a set.  With n_rounds > 1 the candidate arrays (cand, kind,
   * t_req, v_rel, vz0, t_fall) hold n_rounds consecutive rounds of B
   * candidates each, and round r reads the r-th; per-round outputs are
   * overwritten by every round. */
  int32_t n_rounds;      /* 0 or 1: one round; at most FN_MAX_ROUNDS */
  float* incumbent;      /* device [4] or NULL: J*, node* (as float, -1: none), t_best, rounds run.
                          * Initialise to (-inf, -1, t_fall, 0): Algorithm 1 starts with
                          * t_best = t_fall.  When set, a free candidate searches only the
                          * slots with t(parent) + T <= t_best (FP32 sum), every round
                          * replaces the incumbent by its best goal node when that J is
                          * larger, and Prune needs the flight. */
  const float* flight;   /* device [11] or NULL: the object's flight of Eq. (1) for Prune:
                          * x0[3], v0[3], g[3], t_enter, t_fall */
  float* out_reach;      /* device out [ld] or NULL: T_n of Eq. (8) of every node at the last
                          * Prune (before compaction; NaN: no T_n) */
} fn_problem;

#define FN_MAX_ROUNDS 256

typedef struct {
  int32_t n_problems;
  const fn_problem* problems; /* host array */
  int32_t k;
  const float* grid;          /* device [n_t] */
  int32_t n_t, samples, mode; /* mode FN_SEARCH_PLAIN or FN_SEARCH_SCREEN */
  float margin;               /* clearance margin */
  fn_risk risk;
} fn_problem_set;

/* Uploads the problem tables (synchronous).  Sizes and pointers stay fixed
 * until the next prepare; tree contents and node counts are read on the
 * device at every launch.  A graph captured before is discarded (capture
 * again after a prepare).  FN_E_SHAPE beyond max_problems / max_edges /
 * max_batch (sum of B). */
int fn_batch_prepare(fn_ctx* ctx, const fn_problem_set* ps);
/* Enqueues one iteration for the prepared problems: 5 kernels for kNN, the
 * edge search and its FP64 stage, 1 for attachment and scoring. */
int fn_batch_launch(fn_ctx* ctx, void* stream);
/* Captures fn_batch_launch on `stream` into a HIP graph (replaces a
 * previous one); fn_graph_launch replays it.  Memory is cleared by kernels,
 * not memset nodes. */
int fn_graph_capture(fn_ctx* ctx, void* stream);
int fn_graph_launch(fn_ctx* ctx, void* stream);

/* Round `round` (0 .. n_rounds-1) of the prepared problems: the candidates
 * of that round, otherwise as fn_batch_launch (which is round 0). */
int fn_batch_round(fn_ctx* ctx, int32_t round, void* stream);

/* ------------------------------------------------------------------ */
/* Anytime outer loop: arrival-time pruning (Sec. IV-D, Eq. (8)) and   */
/* whole planning cycles (Algorithm 1).                                */
/* ------------------------------------------------------------------ */
typedef struct {
  float v_tip;     /* V_tip of Eq. (8): bound on the blade's speed, m/s (finite, > 0) */
  float blade[3];  /* the blade point p_n, in the frame of the arm's last link, m */
} fn_prune;

/* Earliest reach time of Eq. (8) for n tree nodes (SoA [14][ld], times
 * t_node [n], device): T_n = min{T in [t_enter, t_fall] :
 * t_n + |p_n - x(T)| / V_tip <= T} with x(T) the flight of Eq. (1)
 * (flight: device [11] as in fn_problem); out_T [n] device, NaN where no such
 * T exists.  FP32; a node whose outcome comes close to changing (|G| of the
 * quartic G(T) = |p_n - x(T)|^2 - V_tip^2 (T - t_n)^2 small at a deciding
 * point, a shallow root, or -- in Prune -- T_n within 1 ms of t_best) is
 * recomputed in FP64.  FN_E_ARG for a bad V_tip or blade point. */
int fn_reach_time(fn_ctx* ctx, const float* tree, int64_t ld, int32_t n, const float* t_node,
                  const float* flight, const fn_prune* prune, float* out_T, void* stream);

/* Prune of Algorithm 1 for every prepared problem (all need an incumbent
 * and a flight): a node stays when its T_n exists and T_n <= t_best; node
 * 0, the incumbent and every ancestor of a kept node stay as well.  Kept
 * nodes are compacted in their order (tree, t_node, nu; parents
 * renumbered, freed rows get parent -1), the node count and the
 * incumbent's node index are updated.  Node counts are read on the device. */
int fn_batch_prune(fn_ctx* ctx, const fn_prune* prune, void* stream);

/* One planning cycle of Algorithm 1 for every prepared problem: n_iter
 * anytime iterations of n_round rounds (round a * n_round + r reads
 * candidate round a * n_round + r; n_iter * n_round <= n_rounds), each
 * iteration ending with Prune.  fn_graph_capture_cycle captures the same
 * work into the context's graph (replacing a previous one) for
 * fn_graph_launch. */
int fn_cycle(fn_ctx* ctx, int32_t n_iter, int32_t n_round, const fn_prune* prune, void* stream);
int fn_graph_capture_cycle(fn_ctx* ctx, int32_t n_iter, int32_t n_round, const fn_prune* prune,
                           void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FRUITNINJA_H */
