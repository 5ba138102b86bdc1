// Online-stage kernel of the ReLU-QP solver: the whole loop of Algorithm 1 in one launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rqp {

// Arguments of one persistent solve. Vectors are in the iterate precision T unless noted.
struct LayerArgs {
  int n, m, L;          // L = n + m rows of the compact layer
  long ldw;             // leading dimension of the layer and check matrices (elements)
  const void* W;        // n_rho layer matrices [D, DA'; AD, ADA'] (L x ldw each, T)
  long w_stride;        // elements between consecutive penalty matrices
  const void* C;        // check matrix [P, A'; A, 0] (L x ldw, T)
  const void* q;        // n
  const void* l;        // m
  const void* u;        // m
  const unsigned char* eq;  // m flags: l_i == u_i
  const double* grid;   // n_rho penalty values
  const double* mid;    // n_rho - 1 geometric midpoints between neighbouring grid values
  int n_rho;
  double sigma, alpha, eps_abs, eps_rel, rho_eq_scale;
  int max_iter, check_interval, terminate, warm, j0;
  void* xs;             // handle state x (n), z (m), y (m): read on a warm start, written at exit
  void* zs;
  void* ys;
  int* js;              // handle state penalty index
  int count;            // solves run one after another in this launch (>= 1)
  int chain;            // solves after the first start warm from the previous one
  int max_checks;       // per-solve stride of rho_hist, prim_res, dual_res
  void* xo;             // caller outputs (device), count solves: x count*n, z, y count*m
  void* zo;
  void* yo;
  int* iterations;      // count entries each
  int* status;
  int* rho_index;
  int* rho_hist;        // per check, may be null
  double* prim_res;     // per check, may be null
  double* dual_res;     // per check, may be null
  uint64_t* xw;         // exchange words: layer input, 2 parities x L x words
  uint64_t* xc;         // exchange words: check vector [x; y], 2 x L x words
  uint64_t* xn;         // exchange words: norm partials, 2 x G x 8 x 2
  uint32_t tag;         // first tag of the launch; solve s uses tag + s (max_iter + 2) onwards
  const int* abort_flag;  // host-mapped int, polled at checks
  unsigned* err;        // device word: holds the tag of a solve whose exchange timed out
  int lds_rows;         // rows per block kept in LDS (set by launch_layer from the plan)
  // optional in-kernel update from initial states (x0 != null, count x nx): q = F x0,
  // l = lo - E x0, u = hi - E x0, written to q, l, u before each solve starts
  const double* x0;
  const double* F;      // n x nx
  const double* E;      // m x nx
  const double* plo;    // m
  const double* phi;    // m
  int nx;
};

// Rows per workgroup are at most kMaxRows; the host picks the grid accordingly.
constexpr int kLayerBlock = 1024;
constexpr int kMaxRows = 64;

// Kernel choice and resources for a problem with L = n + m rows on `grid` workgroups: the
// first reg_rows rows of each block stay in registers and the next lds_rows in LDS for the
// whole solve; further rows stream from memory every iteration.
struct LaunchPlan {
  const void* fn;
  int reg_rows, lds_rows;
  size_t dyn_bytes;
  int max_grid;  // largest cooperative grid with these resources
};
template <typename T>
LaunchPlan plan_layer(int L, int grid);

// Launch the persistent solve as a cooperative grid of `grid` workgroups of kLayerBlock threads.
template <typename T>
hipError_t launch_layer(const LayerArgs& a, const LaunchPlan& p, int grid, hipStream_t st);

}  // namespace rqp
