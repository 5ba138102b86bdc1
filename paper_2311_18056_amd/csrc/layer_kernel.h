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
  double* axs;          // handle state A x (m, FP64): the constraint-row owners' carried product
  int warm_ax;          // a warm first solve takes z = A x from axs (the state came from a solve)
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
  int check_cols;       // columns of the check vector staged in LDS at a time (set likewise)
  // optional in-kernel update from initial states (x0 != null, count x nx): q = F x0,
  // l = lo - E x0, u = hi - E x0, written to q, l, u before each solve starts
  const double* x0;
  const double* F;      // n x nx
  const double* E;      // m x nx
  const double* plo;    // m
  const double* phi;    // m
  int nx;
  // optional closed loop (Ad != null, needs x0): solve s starts from the plant state x_s, with
  // x_0 = x0 and x_{s+1} = Ad x_s + Bd u_s, where u_s = z_s[0:nu] + (E x_s)[0:nu] is the first
  // stage's applied control. The owners of constraint rows 0..nu-1 publish u_s in xu
  // (2 parities x nu x 2 words) and every workgroup steps the plant itself, in FP64, in one
  // fixed order (so every copy of x_{s+1} is the same). Trajectories go to traj_x
  // ((count + 1) x nx) and traj_u (count x nu), FP64.
  const double* Ad;     // nx x nx
  const double* Bd;     // nx x nu
  int nu;
  uint64_t* xu;
  double* xpl;          // each workgroup's copy of the plant state: 2 parities x grid x kMaxPlant
  double* traj_x;
  double* traj_u;
  int final_check;      // 0: a max_iter that is not a multiple of check_interval ends unchecked
  // Ruiz scaling (null: none). The kernel iterates on the scaled problem; the check weights
  // each row's terms so that residuals and norms are the original problem's, and the outputs
  // are written unscaled. sc_dual = 1 / (c D) (n), sc_prim = 1 / E (m), un_x = D (n),
  // un_y = E / c (m).
  const double* sc_dual;
  const double* sc_prim;
  const double* un_x;
  const double* un_y;
};

// nx and nu of a closed loop are at most kMaxPlant; grids are at most kMaxGrid workgroups.
constexpr int kMaxPlant = 256;
constexpr int kMaxGrid = 256;

// Rows per workgroup are at most kMaxRows; the host picks the grid accordingly.
constexpr int kLayerBlock = 1024;
constexpr int kMaxRows = 64;

// Split of the residual check over the workgroups. The check reads n L entries of [P, A'] for
// the x rows (dual side) and n m of [A, 0] for the constraint rows (primal side); each
// workgroup forms the constraint rows it owns in the layer (rows split evenly, L / G each), and
// the x rows are split so that every workgroup reads about (n L + n m) / G entries in all.
// split_term(h) is the x-row work (in entries) before workgroup h under that rule; the first x
// row of workgroup g is floor(max_{h <= g} split_term(h) / L), at most n (a running maximum
// keeps the split monotone; g = G gives n). The quotients are formed in double: exact for
// these magnitudes (every product is an integer below 2^53, and a non-integer quotient lies at
// least 1/L from an integer), so host and device agree.
__host__ __device__ inline double split_term(int h, int G, int n, int m, int L) {
  const double total = (double)n * (double)L + (double)n * (double)m;
  const double f = floor((double)h * total / (double)G);
  const int rbase = L / G, rextra = L % G;
  const double r0h = (double)h * rbase + (h < rextra ? h : rextra);
  const double v = f - (double)n * (r0h > n ? r0h - n : 0.0);
  return v > 0.0 ? v : 0.0;
}
__host__ __device__ inline int split_row(double best, int n, int L) {
  const double cb = floor(best / (double)L);
  return cb < (double)n ? (int)cb : n;
}
inline int check_split(int g, int G, int n, int m, int L) {
  double best = 0.0;
  for (int h = 1; h <= g; ++h) {
    const double f = split_term(h, G, n, m, L);
    best = f > best ? f : best;
  }
  return split_row(best, n, L);
}
// The largest share of x rows the split gives a workgroup: at most ceil(L / G) + 1.
constexpr int kMaxCheckRows = kMaxRows + 2;

// Kernel choice and resources for a problem with L = n + m rows on `grid` workgroups: the
// first reg_rows rows of each block stay in registers and the next lds_rows in LDS for the
// whole solve; further rows stream from memory every iteration.
struct LaunchPlan {
  const void* fn;
  int reg_rows, lds_rows;
  int check_cols;  // columns of the check vector staged in LDS at a time
  size_t dyn_bytes;
  int max_grid;  // largest cooperative grid with these resources
};
// xt: the instantiation that also runs closed loops and Ruiz-scaled problems.
template <typename T>
LaunchPlan plan_layer(int L, int grid, bool xt);

// Launch the persistent solve as a cooperative grid of `grid` workgroups of kLayerBlock threads.
template <typename T>
hipError_t launch_layer(const LayerArgs& a, const LaunchPlan& p, int grid, hipStream_t st);

}  // namespace rqp
