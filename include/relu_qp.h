/*
 * relu_qp.h -- C ABI of the MI355X (gfx950) ReLU-QP solver.
 *
 * Solves the convex QP of arXiv 2311.18056, Sec. II-A (eq. qp_def):
 *
 *     minimise 1/2 x'Px + q'x   subject to   l <= A x <= u,
 *
 * with the ADMM iteration recast as a weight-tied layer (Sec. III-A, eq. gpu_update) and run
 * as in Algorithm 1: an offline stage that forms the KKT inverse
 * D_j = (P + sigma I + A' diag(rho_j) A)^-1 for every penalty value rho_j of a fixed grid
 * (Sec. III-C, penalty heuristics), and an online stage that repeats "matvec, clamp, dual
 * update" with a residual check (eqs. primal, dual) and a penalty switch (eq. rho_update)
 * every check_interval iterations (Sec. III-C, convergence checking).
 *
 * Letters follow OSQP: the paper's (H, g, G, c, d) are (P, q, A, l, u); its primal y is x, its
 * constraint copy z is z, and its multiplier lambda is y.
 *
 * Conventions for every function:
 *   - return value: RQP_OK (0) or a negative RQP_E* code; nothing else crosses the ABI;
 *     relu_qp_last_error() gives a message for the calling thread's last failure;
 *   - matrices are dense, row-major, FP64, on the HOST unless the name says "device";
 *   - inputs are borrowed for the duration of the call only (the library copies them);
 *   - a handle owns all device memory it allocates and is not thread-safe; distinct handles
 *     are independent;
 *   - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 */
#ifndef RELU_QP_H
#define RELU_QP_H

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
enum {
  RQP_OK = 0,
  RQP_EINVAL = -1, /* bad argument: sizes, non-finite P or A, asymmetric P, l > u, settings */
  RQP_ENOMEM = -2, /* device allocation failed */
  RQP_EHIP = -3,   /* a HIP runtime call failed (message from relu_qp_last_error) */
  RQP_ENOTPD = -4, /* P + sigma I + A' diag(rho) A is not positive definite for some rho */
  RQP_ESTATE = -5  /* NULL handle, or a call out of order */
};

/* per-instance solver status written by relu_qp_solve (Algorithm 1's loop exits) */
enum {
  RQP_RUNNING = 0,
  RQP_SOLVED = 1,    /* r_p <= eps_p and r_d <= eps_d at a check (eqs. primal, dual) */
  RQP_MAX_ITER = 2,  /* max_iter reached (also for infeasible problems: no detection) */
  RQP_NONFINITE = 3, /* a residual norm was NaN or infinite */
  RQP_ABORTED = 4,   /* relu_qp_abort() was seen at a check */
  RQP_INTERNAL = 5,  /* the in-kernel exchange timed out (a library fault, never expected) */
  RQP_IDLE = 6       /* serving: the slot holds no instance */
};

/* arithmetic of the online iteration */
enum {
  RQP_FP64 = 0,  /* FP64 weights, iterates and residuals (single-instance engine) */
  RQP_FP32 = 1,  /* FP32 weights and iterates; single-instance engine: residual products
                    accumulated in FP64; batched engine: FP32 matrix-core products */
  RQP_BF16X3 = 2 /* batched engine: weights and layer inputs split into BF16 high + low parts,
                    three BF16 matrix-core products (hi*hi + lo*hi + hi*lo) accumulated in FP32,
                    FP32 iterates, FP64 residual norms */
};

/* which kernel runs the online stage */
enum {
  RQP_ENGINE_AUTO = 0,   /* single-instance for batch == 1 with FP64/FP32, else batched */
  RQP_ENGINE_SINGLE = 1, /* one instance spread over the whole GPU (batch must be 1) */
  RQP_ENGINE_BATCH = 2   /* many instances as one GEMM per iteration (FP32 or BF16X3) */
};

typedef struct {
  double sigma;        /* proximal weight sigma > 0 (Sec. II-B); default 1e-6 */
  double alpha;        /* over-relaxation in (0, 2); 1 gives the paper's iteration; default 1.6 */
  double rho0;         /* initial penalty (Sec. III-C: 0.1); the grid value nearest in log */
  int n_rho;           /* 1: fixed penalty rho0; >1: log grid rho_min..rho_max (default 1) */
  double rho_min;      /* default 1e-3 */
  double rho_max;      /* default 1e3 */
  double rho_eq_scale; /* penalty factor on rows with l_i == u_i (Sec. II-B: 1000) */
  double eps_abs;      /* eps = eps_abs + eps_rel * max(norms); both 0: run exactly max_iter */
  double eps_rel;
  int max_iter;        /* default 4000 */
  int check_interval;  /* default 25 (Sec. III-C); a check also runs at max_iter */
  int precision;       /* RQP_FP64, RQP_FP32 or RQP_BF16X3 */
  int batch;           /* instances sharing P and A (>= 1) */
  int engine;          /* RQP_ENGINE_* (default AUTO) */
  int scaling;         /* passes of the modified Ruiz equilibration with cost scaling (Algorithm 1
                        * "scale problem", Sec. III-D; OSQP's form): 0 (default) = none, at most
                        * 100. The solve iterates on the scaled problem; termination, residuals
                        * and outputs are in the original units. On the batched engine one
                        * scaling serves the batch (its cost scale from the largest |q| entry
                        * over the setup instances); closed loops run unscaled. */
} relu_qp_settings;

typedef struct relu_qp_handle relu_qp_handle; /* opaque, library-owned */

/* Caller-owned DEVICE buffers the solve writes, asynchronously on its stream.
 * x: batch*n, y (dual) and z: batch*m, in the iterate precision (double for RQP_FP64,
 * float for RQP_FP32), instance-major. iterations, status, rho_index: batch ints.
 * rho_hist (ints), prim_res and dual_res (doubles): batch * relu_qp_max_checks() entries,
 * one per check (grid index in force after the check, r_p, r_d); each may be NULL. */
typedef struct {
  void* x;
  void* y;
  void* z;
  int* iterations;
  int* status;
  int* rho_index;
  int* rho_hist;
  double* prim_res;
  double* dual_res;
} relu_qp_result;

/* Fills *s with the defaults above. */
void relu_qp_default_settings(relu_qp_settings* s);

/* Offline stage of Algorithm 1 (Sec. III-B): validates the problem, copies it to the device
 * and forms, in FP64 on the GPU, the layer weights of every grid penalty.
 *   P: n*n symmetric positive semidefinite; A: m*n; q: batch*n; l, u: batch*m, -/+INFINITY
 *   allowed, l <= u. The equality-row pattern (l_i == u_i) is taken from the first instance.
 * Synchronises before returning (it must report RQP_ENOTPD). On success *h is a new handle;
 * on failure *h is NULL and nothing is leaked. */
int relu_qp_setup(relu_qp_handle** h, int n, int m, const double* P, const double* q, const double* A,
                  const double* l, const double* u, const relu_qp_settings* s, void* stream);

/* Online stage, "update b, c~, d~" of Algorithm 1: new q (batch*n), l, u (batch*m) from the
 * host; NULL leaves a vector unchanged. RQP_EINVAL if l > u or the equality-row pattern
 * changes (the weights depend on it). Synchronous. */
int relu_qp_update(relu_qp_handle* h, const double* q, const double* l, const double* u);

/* Same, from DEVICE FP64 buffers, asynchronously on stream; no validation of l <= u. */
int relu_qp_update_device(relu_qp_handle* h, const double* q, const double* l, const double* u, void* stream);

/* Parametric (MPC) data, Sec. IV: q = F x0, l = lo - E x0, u = hi - E x0 with F (n*nx) and
 * E (m*nx) row-major. Copies F, E, lo, hi to the device. Synchronous. */
int relu_qp_set_parametric(relu_qp_handle* h, int nx, const double* F, const double* E, const double* lo,
                           const double* hi);

/* Online update from initial states: x0 is a DEVICE FP64 array of batch*nx values; computes
 * q, l, u of every instance on the GPU, asynchronously on stream. */
int relu_qp_update_x0_device(relu_qp_handle* h, const double* x0, void* stream);

/* Warm start (Sec. II-B): the next solve starts from x (batch*n), y (batch*m) and grid index
 * rho_index (the same for every instance), with z = A x. Host FP64 arrays. Synchronous. */
int relu_qp_warm_start(relu_qp_handle* h, const double* x, const double* y, int rho_index);

/* enabled != 0: every later solve starts from the previous solve's x, y and penalty, with
 * z = A x (the receding-horizon use of Sec. V-B). 0 (the default): cold starts. */
int relu_qp_set_warm(relu_qp_handle* h, int enabled);

/* Online loop of Algorithm 1, asynchronously on stream: one kernel launch (the persistent grid,
 * or one workgroup when n + m <= 128; see relu_qp_set_launch) runs every iteration, check and
 * penalty switch. Results go to out (caller-owned device buffers); read them after a stream
 * synchronisation. */
int relu_qp_solve(relu_qp_handle* h, void* stream, relu_qp_result* out);

/* relu_qp_update_x0_device followed by relu_qp_solve, in one launch for the single-instance
 * engine (the kernel forms q, l, u of its rows from x0 before iterating, with the same FP64
 * products, and writes them back). x0: DEVICE FP64, batch*nx. RQP_ESTATE without parametric
 * data. */
int relu_qp_solve_x0(relu_qp_handle* h, const double* x0, void* stream, relu_qp_result* out);

/* `count` solves one after another in ONE launch of the single-instance engine, solve s from
 * initial state x0s[s*nx ..] (DEVICE FP64, count*nx). The layer weights stay on chip between
 * the solves. Solve s writes its results at index s of out: x at s*n, y and z at s*m,
 * iterations/status/rho_index at s, rho_hist/prim_res/dual_res at s*relu_qp_max_checks().
 * The first solve starts as relu_qp_solve would; with relu_qp_set_warm(h, 1) each later solve
 * starts warm from the previous one (the receding-horizon use), else cold. Needs parametric
 * data; RQP_EINVAL if count < 1, on the batched engine, or count*(max_iter+2) >= 2^31. */
int relu_qp_solve_sequence(relu_qp_handle* h, const double* x0s, int count, void* stream, relu_qp_result* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, hosts that forbid hipMalloc at run time): relu_qp_solve_x0 with the launch's scratch
 * (the exchange words of the layer input, the check vector and the norm partials, and the
 * error word) in a device array inside the library instead of the handle's allocations. The
 * call allocates nothing, frees nothing and issues no memset (the scratch is cleared by a
 * kernel on first use on a GPU and whenever its tag sequence restarts). The array holds
 * 1 MiB on each GPU the library runs on (enough for every n + m the single-instance engine
 * accepts; RQP_EINVAL otherwise) and stays until the process ends. Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams, other threads) race, so
 * serialise them. Same arguments, results and handle state as relu_qp_solve_x0; the current
 * device must be the one the handle was set up on (RQP_ESTATE otherwise, also on the batched
 * engine). */
int relu_qp_solve_x0_noalloc(relu_qp_handle* h, const double* x0, void* stream, relu_qp_result* out);

/* The paper's literal layer (eq. gpu_update), for comparison with the compact form the solver
 * runs: v <- clamp(W v + b, c~, d~) with v = [x; z; lambda] (n + 2m), W the full
 * (n+2m) x (n+2m) weight matrix built from the handle's matrices at first use (FP64 products,
 * stored in the iteration precision, streamed from memory every layer), b = [-D q; -A D q; 0]
 * from the handle's q, only the z block clamped to [l, u]. Runs `iters` layers from v = 0 in
 * one launch, asynchronously on stream, and writes x, z and the lagged dual lambda (the
 * textbook dual of the previous layer) to out->x, out->z, out->y; iterations = iters, status
 * RQP_MAX_ITER. Exactly the textbook iteration at alpha = 1 with a fixed penalty, so it needs
 * alpha == 1 and n_rho == 1 (RQP_EINVAL otherwise, or with Ruiz scaling, iters outside
 * [1, 2^24], or n + 2m > 16384); RQP_ESTATE on the batched engine. The weights (and their
 * exchange words) stay allocated with the handle after the first call. */
int relu_qp_solve_paper_form(relu_qp_handle* h, int iters, void* stream, relu_qp_result* out);

/* Closed-loop MPC (the receding-horizon use of Sec. V-B) in ONE launch of the single-instance
 * engine: `steps` MPC steps, step s from the plant state x_s (x_0 = x0, DEVICE FP64, nx):
 * q, l, u from x_s as in relu_qp_solve_x0, then settings.max_iter iterations (the per-step
 * budget; a budget that is not a multiple of check_interval ends without a check, status
 * RQP_MAX_ITER; with eps > 0 a check may also end a step early), warm from the previous step
 * (x, y and penalty index; z = A x) — the first step starts as relu_qp_solve would — then
 * the applied control u_s = z[0:nu] + (E x_s)[0:nu] (the first nu constraint rows hold the
 * first stage's control, as the condensed form lays them out) and the plant step
 * x_{s+1} = Ad x_s + Bd u_s, all on the device.
 * Ad: nx*nx, Bd: nx*nu row-major (DEVICE FP64); traj_x: (steps+1)*nx, traj_u: steps*nu
 * (DEVICE FP64, caller-owned, written asynchronously on stream); out: results of each step at
 * index s as in relu_qp_solve_sequence. Needs parametric data (RQP_ESTATE); RQP_EINVAL for
 * NULL pointers, steps < 1, nu outside [1, min(m, 256)], nx > 256, or a handle with Ruiz
 * scaling; RQP_ESTATE on the batched engine. relu_qp_abort is seen at checks only, so a loop
 * whose budget stays below check_interval runs all its steps. */
int relu_qp_closed_loop(relu_qp_handle* h, const double* x0, int steps, const double* Ad, const double* Bd, int nu,
                        double* traj_x, double* traj_u, void* stream, relu_qp_result* out);

/* ---- Serving (continuous batching; batched engine only).
 * The handle's `batch` instances are slots. A slot holds one request from its admission until
 * a final status; finished and idle slots cost nothing in a step. Warm starts follow the
 * receding-horizon use of Sec. II-B / V-B: the last solution of the same QP family, shifted
 * by one stage. All four calls are asynchronous on stream; `slots` is a HOST array of
 * n_slots distinct indices in [0, batch). */

/* q, l, u of the listed slots from DEVICE FP64 rows (n_slots*n, n_slots*m); NULL keeps a
 * vector. No validation of l <= u. */
int relu_qp_load_slots(relu_qp_handle* h, const int* slots, int n_slots, const double* q, const double* l,
                       const double* u, void* stream);

/* q, l, u of the listed slots from initial states x0 (DEVICE FP64, n_slots*nx) with the
 * parametric data of relu_qp_set_parametric (Sec. IV). */
int relu_qp_load_slots_x0(relu_qp_handle* h, const int* slots, int n_slots, const double* x0, void* stream);

/* The listed slots start at the next relu_qp_step: cold (src_slot == -1: x = z = y = 0 and the
 * start penalty), or warm from the current x and y of slot src_slot shifted forward by
 * shift_x and shift_y entries (entries shifted in from beyond the end are 0; the stage-major
 * layout of Sec. IV makes one stage nu entries), with its penalty index and z = A x. The
 * source is read before any listed slot is written, so it may be one of them. */
int relu_qp_admit(relu_qp_handle* h, const int* slots, int n_slots, int src_slot, int shift_x, int shift_y,
                  void* stream);

/* One persistent launch of at most n_checks * check_interval iterations for every running or
 * admitted slot. Slots stop at checks exactly as in relu_qp_solve; iterations count from
 * admission, so a slot reaches max_iter across several steps. Afterwards every slot's x, y, z,
 * status (RQP_RUNNING while unfinished), iterations and rho_index are in out; rho_hist,
 * prim_res and dual_res entries are written at index (check number since admission).
 * Needs max_iter % check_interval == 0 (RQP_EINVAL otherwise). */
int relu_qp_step(relu_qp_handle* h, int n_checks, void* stream, relu_qp_result* out);

/* Tile shape of the batched engine's GEMM: 128, 64 or 256 matrix rows per tile (x 128 instances);
 * with 128 or 256, the last that many rows of the layer go in tiles of half the rows, run last.
 * relu_qp_setup of a batched handle runs an autotuner: every shape runs two check intervals of
 * all slots on the handle's own data, timed on the device, and the fastest is kept, where a
 * shape later in the order 128, 64, 256 must be more than 1 % faster than an earlier one (slots
 * are idle and the state zero afterwards). The choice and timings are cached for the rest of the
 * process per device and problem shape (n, m, batch, precision, number of penalties): a later
 * handle of the same shape (a family loaded again) takes them without timing. The shapes
 * agree to rounding (the same products per element, issued to the matrix cores in another
 * interleaving).
 * relu_qp_get_tile: the shape in use and, in us_per_iter[3] (may be NULL), the autotuner's
 * microseconds per iteration for 128, 64 and 256 rows. relu_qp_set_tile: force 128, 64 or 256,
 * or 0 for the autotuner's choice. RQP_ESTATE on a single-instance handle. */
int relu_qp_get_tile(const relu_qp_handle* h, int* tile_rows, double* us_per_iter);
int relu_qp_set_tile(relu_qp_handle* h, int tile_rows);

/* Device memory, for admission by memory (a server keeps problem families resident in HBM
 * while their sizes fit a budget).
 * relu_qp_device_bytes: the bytes the handle holds now (requested sizes of its resident
 * allocations: layer and check weights for every penalty, state, operand and exchange buffers,
 * parametric data). RQP_ESTATE on NULL.
 * relu_qp_footprint: the same figure for a handle that relu_qp_setup(n, m, s) would create,
 * plus F, E, lo, hi if nx > 0 (relu_qp_set_parametric), computed on the host without any
 * device call; *setup_extra (may be NULL) receives the FP64 workspace setup holds on top of
 * that while it factors. RQP_EINVAL for bad sizes or settings (as relu_qp_setup). */
int relu_qp_device_bytes(const relu_qp_handle* h, size_t* bytes);

/* Spill and restore, so that a server can take a family out of HBM without losing its setup:
 * relu_qp_offload waits for the device, copies every resident allocation of the handle
 * (weights, state, slots, exchange words) to pinned host memory (allocated at the first
 * offload and kept with the handle) and frees the device memory: relu_qp_device_bytes then
 * reports 0, and every call that needs the device returns RQP_ESTATE. relu_qp_restore
 * allocates the device memory again and copies everything back, so the handle continues
 * exactly where it stopped. Both are synchronous; a second offload (restore) is a no-op.
 * RQP_ENOMEM if the host (device) memory cannot be had; the handle is then left as it was. */
int relu_qp_offload(relu_qp_handle* h);
int relu_qp_restore(relu_qp_handle* h);
int relu_qp_footprint(int n, int m, const relu_qp_settings* s, int nx, size_t* bytes, size_t* setup_extra);

/* Ask a running solve to stop with status RQP_ABORTED (any thread). The flag lives in host
 * memory and a kernel polls it at every 16th check of a launch (every 400 iterations with the
 * default check_interval), since each poll is a PCIe round trip. */
int relu_qp_abort(relu_qp_handle* h);

/* Sizes of the result arrays and the grid. */
int relu_qp_max_checks(const relu_qp_handle* h);
int relu_qp_get_rho_grid(const relu_qp_handle* h, double* grid /* n_rho */, int* n_rho);

/* Launch shape of the single-instance solves. By default (grid 0) a problem with
 * n + m <= 128 runs its solves (relu_qp_solve, relu_qp_solve_x0, relu_qp_solve_sequence) on one
 * workgroup with the layer matrix in registers; larger problems run the persistent kernel on
 * about one workgroup per 12.5 rows (fewer when a workgroup holds fewer rows on chip, at most
 * one per compute unit), and closed loops and Ruiz-scaled problems on one workgroup per compute
 * unit (at most one per row).
 * A grid > 0 makes every solve use the persistent kernel on that many workgroups; it must lie
 * in [ceil((n+m)/64), min(n+m, the cooperative limit)]. relu_qp_get_launch reports the grid of
 * plain solves (1 for the single-workgroup kernel) and the workgroup size. */
int relu_qp_set_launch(relu_qp_handle* h, int grid);
int relu_qp_get_launch(const relu_qp_handle* h, int* grid, int* block);

/* Frees everything the handle owns; NULL is a no-op. Synchronises the device. */
int relu_qp_cleanup(relu_qp_handle* h);

/* Message of the calling thread's last failed call ("" if none). Never NULL. */
const char* relu_qp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RELU_QP_H */
