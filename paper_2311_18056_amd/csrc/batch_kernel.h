// Batched online stage: many instances that share P and A (so the layer matrices), each with
// its own q, l, u, state, penalty index and termination, in one persistent launch. The layer
// product of all active instances is a GEMM on the matrix cores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rqp {

enum BatchPrec { kBatchF32 = 0, kBatchBF16x3 = 1 };

// Slot states beyond the public statuses: a slot is idle until admitted; an admitted slot
// starts at the next launch, cold (x = z = y = 0, start penalty) or warm (x, y and penalty
// index already in place, z = A x).
enum { kSlotIdle = 6, kSlotAdmitCold = 16, kSlotAdmitWarm = 17 };

// Up to 64 slot indices passed by value in the kernel arguments.
constexpr int kMaxSlotsPerCall = 64;
struct SlotList {
  int n;
  int s[kMaxSlotsPerCall];
};

constexpr int kTileM = 128;   // instances per tile
constexpr int kTileN = 256;   // layer rows per tile (largest tile shape; 128 and 64 also exist)
constexpr int kTileK = 32;    // k per LDS stage
constexpr int kBatchBlock = 256;

struct BatchArgs {
  int n, m, L, B;
  // K-blocked layout of every GEMM operand: element (row, c) of a matrix with `rows` padded
  // rows is at ((c / kTileK) * rows + row) * kTileK + c % kTileK, so one K stage of a tile is
  // one contiguous block. ldk = columns (multiple of kTileK, with zero padding).
  long ldk;
  long lpad;                // padded rows of the layer matrices (multiple of kTileN)
  long cpad;                // padded rows of the check matrix (at least L + 128: constraint-row
                            // tiles start at row n)
  long bpad;                // padded rows (list positions) of the operands V and CV
  int prec;                 // BatchPrec
  const void* Wa;           // FP32 layer matrices, or BF16 high parts: n_rho blocked lpad x ldk
  const void* Wb;           // BF16 low parts (kBatchBF16x3), else null
  long w_stride;            // elements between penalty matrices
  const double* Cd;         // check matrix [P, A'; A, 0] in FP64, same format (blocked cpad x ldk);
                            // with Ruiz scaling the original (unscaled) P and A
  const float* Q;           // B x n
  const float* Lo;          // B x m
  const float* Up;          // B x m
  // Ruiz scaling (null: none). The layer runs on the scaled problem (x = D xb, z = zb / E,
  // y = E yb / c); Q, Lo, Up hold c D q, E l, E u. Layout: c D (n), E (m), 1 / (c D) (n),
  // 1 / E (m), D (n), E / c (m). The check evaluates the original problem at the unscaled
  // iterates rounded to FP32 exactly as the outputs are (unscale_outputs).
  const double* scl;
  const unsigned char* eq;  // m
  const double* grid;
  const double* mid;
  int n_rho;
  double sigma, alpha, eps_abs, eps_rel, rho_eq_scale;
  int max_iter, check_interval, terminate, j0;
  int steps;                // iterations this launch may run (max_iter for a whole solve)
  float* X;                 // state B x n
  float* Z;                 // state B x m
  float* Y;                 // state B x m
  // operand rows are list positions (the bucketed order of the running instances), so a tile's
  // rows are contiguous
  void* Va;                 // layer inputs, 2 parities x blocked bpad x ldk (FP32, or BF16 high)
  void* Vb;                 // BF16 low parts
  double* CVd;              // check operands in FP64 (exact copies of the FP32 iterates, unscaled as the
                            // outputs are), two blocked bpad x ldk arrays: [x; 0], then [0; y] (the
                            // zeros are never written)
  double* Rpx;              // B x n: P x of list position p in row p (check scratch)
  double* Raty;             // B x n: A'y likewise
  int* jb;                  // B penalty indices (kept for running and warm-admitted slots)
  int* status;              // B slot states (kSlot* below, or a final status), persistent
  int* iterations;          // B iterations since admission, persistent
  int* rho_hist;            // B x max_checks, may be null
  double* prim_res;         // B x max_checks, may be null
  double* dual_res;         // B x max_checks, may be null
  int max_checks;
  unsigned long long* norms;  // B x 8 (ordered FP64 bit patterns), zero at launch
  int* lists;               // B instance ids grouped by penalty index
  int* pos_of;              // B list position of each running instance
  int* mtiles;              // per M-tile: {j, offset, count}, up to B/kTileM + n_rho entries, + count
  unsigned* bar;            // grid barrier words (zero at launch)
  const int* abort_flag;    // host-mapped
};

struct BatchPlan {
  const void* fn;
  int grid;
  size_t smem;
  int tn;  // matrix rows per tile (256, 128 or 64)
};

// Kernel of the given precision and tile rows (256, 128 or 64); fn == null if unavailable.
constexpr int kTileShapes = 3;
constexpr int kTileRows[kTileShapes] = {128, 64, 256};
BatchPlan plan_batch(int prec, int tn);
// Set every slot's state (e.g. admit all for a whole-batch solve).
hipError_t fill_status(int B, int value, int* status, hipStream_t st);
// q, l, u of the listed slots: from initial states x0 (n_slots x nx, FP64, device) with the
// parametric data F, E, lo, hi; or copied from FP64 device rows (a NULL vector is kept).
hipError_t load_x0_slots(const SlotList& sl, int n, int m, int nx, const double* F, const double* E, const double* lo,
                         const double* hi, const double* x0, float* Q, float* Lo, float* Up, hipStream_t st);
// With Ruiz scaling (scl != null) the copied rows are scaled on the way (c D q, E l, E u); the
// parametric data of load_x0_slots is scaled once at set-up instead.
hipError_t load_slots(const SlotList& sl, int n, int m, const double* q, const double* l, const double* u, float* Q,
                      float* Lo, float* Up, const double* scl, hipStream_t st);
// Admit the listed slots: cold (src == -1), or warm from slot src's x and y shifted by sx / sy
// entries (entries shifted in from beyond the end are 0) and its penalty index. The source is
// first copied to stage (n + m floats and one int); src == -2 reuses what stage holds. With Ruiz
// scaling (scl != null) a shifted entry moves to another row's units: x_i <- x_{i+sx} D_{i+sx} / D_i,
// y_i <- y_{i+sy} (E/c)_{i+sy} / (E/c)_i (an unshifted copy stays exact).
hipError_t admit_slots(const SlotList& sl, int src, int sx, int sy, int n, int m, float* X, float* Y, int* jb,
                       int* status, float* stage, const double* scl, hipStream_t st);
// Outputs in original units from the scaled state: x = D xb, z = zb (1 / E), y = yb (E / c), each
// rounded to FP32 from the FP64 product (the values the check evaluated).
hipError_t unscale_outputs(int B, int n, int m, const float* X, const float* Z, const float* Y, const double* scl,
                           float* x, float* z, float* y, hipStream_t st);
hipError_t launch_batch(const BatchArgs& a, const BatchPlan& p, hipStream_t st);

// FP64 row-major rows x cols -> K-blocked lpad x ldk (zero padded): BF16 high and low parts,
// or FP32.
hipError_t split_bf16(long rows, int cols, const double* src, long ld_src, void* hi, void* lo, long lpad, long ldk,
                      hipStream_t st);
hipError_t pad_f32(long rows, int cols, const double* src, long ld_src, float* dst, long lpad, long ldk,
                   hipStream_t st);
hipError_t pad_f64(long rows, int cols, const double* src, long ld_src, double* dst, long lpad, long ldk,
                   hipStream_t st);
// Dynamic LDS bytes of the batched kernel with this plan (the larger of its GEMM tile stages).
size_t batch_smem(int prec, int tn);

}  // namespace rqp
