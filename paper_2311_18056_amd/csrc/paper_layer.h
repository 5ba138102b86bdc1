// The paper's literal weight-tied layer (eq. gpu_update): v <- clamp(W v + b, c~, d~) with
// v = [x; z; lambda] (n + 2m entries, lambda the dual lagged by one step), the full
// (n+2m) x (n+2m) weight matrix W and b = [-D q; -A D q; 0]; only the z block is clamped.
// It equals the textbook iteration at alpha = 1 with a fixed penalty (the dual shifted by one
// step). Kept as an ablation of the compact form the solver runs: 2.25x the weight bytes of
// the compact matrix at m = n, streamed every iteration, one exchange per iteration as well.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rqp {

constexpr int kPaperBlock = 1024;
constexpr int kPaperMaxRows = 64;      // rows per workgroup
constexpr int kPaperMaxL = 16384;      // n + 2m (the layer input lives in LDS, padded to ldp)

struct PaperArgs {
  int n, m, Lp;           // Lp = n + 2m
  long ldp;               // leading dimension of W (elements)
  const void* W;          // Lp x ldp, iteration precision T
  const void* Wc;         // compact layer matrix (L x ldw, T); its first n columns are [D; A D]
  long ldw;
  const void* q;          // n, T
  const void* l;          // m, T
  const void* u;          // m, T
  int iters;
  uint64_t* xw;           // exchange words: 2 parities x Lp x words
  uint32_t tag;           // tags tag + 1 .. tag + iters
  unsigned* err;          // device word: the tag of a launch whose exchange timed out
  void* xo;               // outputs (T): x (n), z (m), the lagged dual (m)
  void* zo;
  void* yo;
  int* iterations;
  int* status;
};

// W = the paper's weight matrix for penalty vector rho (m), from the compact matrix of the same
// penalty (D, D A', A D, A D A') and A (the check matrix's lower-left block), via two FP64
// products (D A') diag(rho) A and (A D A') diag(rho) A. W: Lp x ldp in T.
template <typename T>
hipError_t assemble_paper_w(int n, int m, const T* Wc, long ldw, const T* C, const double* rho, double sigma, T* W,
                            long ldp, hipStream_t st);

// One persistent cooperative launch of `grid` workgroups running a.iters layers from v = 0.
template <typename T>
hipError_t launch_paper_layer(const PaperArgs& a, int grid, hipStream_t st);

}  // namespace rqp
