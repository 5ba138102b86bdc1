// Single-workgroup ReLU-QP kernel for small problems (n + m <= 128): every iteration, check and
// penalty switch of Algorithm 1 (online stage) in one launch of one workgroup.
//
// The iteration is the compact layer of the persistent kernel (Sec. III-A with OSQP
// over-relaxation): w = [sigma x - q ; rho z - y], one product with
// Wc_j = [D_j, D_j A'; A D_j, A D_j A'] gives xt and A xt, and the relaxation, the clamp
// (eq. clamp) and the dual update are row-local. At these sizes an iteration is a few hundred
// multiply-adds, so its time is set by latency, not by bandwidth: a persistent grid would spend
// it on the cross-workgroup exchange of w. Here Wc_j lives in registers for the whole solve
// (reloaded when the penalty changes), w is exchanged through LDS, and one workgroup barrier per
// iteration is the only synchronisation.
//
// Layout: row r of Wc_j is split over S = 8 consecutive lanes;
// lane s of the row holds and multiplies the columns c = s, s + S, ... (at most 16 values) and
// DPP lane moves sum the S partials, leaving the row's value in all S lanes. Waves that hold
// no row skip the product.
//
// Every check_interval iterations (Sec. III-C) the rows of [P, A'; A, 0] [x; y] (P x + A'y and
// A x) are formed with FP64 accumulation from the check matrix, held in LDS for the whole
// launch, and the seven inf-norms are reduced as ordered bit patterns (exact and
// NaN-propagating). The stopping test (eqs. primal, dual) and
// the penalty rule (eq. rho_update, nearest grid value) are those of the persistent kernel.
#include "small_kernel.h"

#include "device_common.h"

namespace rqp {
namespace {

constexpr int SB = kSmallBlock;
constexpr int SWAVES = SB / kWave;
constexpr int kRhoMax = 64;  // the host accepts at most 64 penalty values

enum { S_RUNNING = 0, S_SOLVED = 1, S_MAX_ITER = 2, S_NONFINITE = 3, S_ABORTED = 4 };
enum { K_RP = 0, K_RD, K_AX, K_Z, K_PX, K_ATY, K_Q, K_NORMS };

// Shapes: S lanes per row and NI column blocks (columns c = i S + s, zero past L): S = 8 (a wave
// holds 8 rows) and NI = 8, 12 or 16 for L <= 64, 96 or 128. For L <= 64, 8 x 8 measured 2 %
// faster than 16 lanes x 4 blocks (one DPP step less per row sum) and 25 % faster than 4 x 16.
constexpr int kBatch = 4;  // loads issued together (NI is a multiple)
__host__ __device__ constexpr int small_lanes(int) { return 8; }
__host__ __device__ constexpr int small_blocks(int L) { return L <= 64 ? 8 : (L <= 96 ? 12 : 16); }

// Sum over the S lanes of a row (S in 1, 2, 4, 8, 16; the lanes are consecutive and S-aligned)
// with DPP lane moves (VALU, no LDS round trip): swaps of neighbours and of pairs within a quad,
// then the half-row and row mirrors. Every lane of the row ends with the same sum (each step
// adds the same two partial sums, in either order).
template <int S, typename T>
__device__ __forceinline__ T row_sum(T v) {
  if constexpr (S >= 2) v = dpp_add<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  if constexpr (S >= 4) v = dpp_add<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  if constexpr (S >= 8) v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  if constexpr (S >= 16) v = dpp_add<0x140, 0xf>(v); // row_mirror
  return v;
}

// This lane's entries of row r of the layer matrix of penalty j: W[r][i S + s], i < NI (zero
// for rows or columns past L). Lanes of a row read consecutive columns.
template <typename T, int S, int NI>
__device__ __forceinline__ void load_row(const LayerArgs& a, int j, bool row, int r, int s, T (&wst)[NI]) {
  const T* Wr = static_cast<const T*>(a.W) + (long)j * a.w_stride + (long)(row ? r : 0) * a.ldw;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int c = i * S + s;
    wst[i] = (row && c < a.L) ? Wr[c] : (T)0;
  }
}

// The check matrix [P, A'; A, 0] into LDS as [i][t]: thread t = r S + s finds C[r][i S + s] at
// i * 1024 + t (zero for rows or columns past L). Loaded once per launch.
template <typename T, int S, int NI>
__device__ void load_check(const LayerArgs& a, T* Cl) {
  const T* Cm = static_cast<const T*>(a.C);
  const int L = a.L;
  for (int e = threadIdx.x; e < NI * SB; e += SB) {
    const int i = e / SB, t = e - i * SB, r = t / S, c = i * S + (t - r * S);
    Cl[e] = (r < L && c < L) ? Cm[(long)r * a.ldw + c] : (T)0;
  }
}

// Products of this lane's part of its row of the check matrix with cv over the columns
// c = i S + s < cend, FP64, split at column n (the P or A part and the A' part), accumulated in
// ascending column order, with the sums of their absolute values (alo, ahi: the rounding bound
// of the check); columns out of range contribute zero.
template <typename T, int S, int NI>
__device__ __forceinline__ void check_products(const LayerArgs& a, const T* Cl, int s, int cend, const T* cv,
                                               double& lo, double& hi, double& alo, double& ahi) {
  lo = 0.0;
  hi = 0.0;
  alo = 0.0;
  ahi = 0.0;
#pragma unroll
  for (int i0 = 0; i0 < NI; i0 += kBatch) {
    T cval[kBatch], xval[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      cval[b] = Cl[(i0 + b) * SB + threadIdx.x];
      xval[b] = cv[(i0 + b) * S + s];
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int c = (i0 + b) * S + s;
      const double v = c < cend ? (double)cval[b] * (double)xval[b] : 0.0;
      if (c < a.n) {
        lo += v;
        alo += fabs(v);
      } else {
        hi += v;
        ahi += fabs(v);
      }
    }
  }
}

template <typename T, int S, int NI>
__global__ void __launch_bounds__(SB) small_kernel(LayerArgs a) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  T* Cl = reinterpret_cast<T*>(dyn_lds);  // the check matrix, NI * 1024 entries
  __shared__ T wb[2][kSmallRows];   // layer input w, two parities
  __shared__ T cv[kSmallRows];      // [x; y] for the check and z = A x of a warm start
  __shared__ T upd[kSmallRows][2];  // q, l, u from an initial state
  __shared__ uint64_t nrm[K_NORMS][kSmallRows];
  __shared__ uint64_t fin[K_NORMS + 1];
  __shared__ double grid_s[kRhoMax], mid_s[kRhoMax];
  __shared__ int decision[2];

  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int n = a.n, L = a.L;
  const int r = tid / S, s = tid - r * S;  // this lane's row and column lane
  const bool wave_rows = wave * (kWave / S) < L;  // the wave holds at least one row
  const bool row = r < L, own = row && s == 0, xrow = r < n;
  const bool seq = row && !xrow && a.eq[r - n] != 0;

  if (tid < a.n_rho) grid_s[tid] = a.grid[tid];
  if (tid < a.n_rho - 1) mid_s[tid] = a.mid[tid];
  // entries past L are read as columns of the zero padding; keep them finite
  if (tid < kSmallRows && tid >= L) wb[0][tid] = wb[1][tid] = cv[tid] = (T)0;
  load_check<T, S, NI>(a, Cl);

  const int ci = a.check_interval, max_iter = a.max_iter;
  const T alpha = (T)a.alpha, oma = (T)(1.0 - a.alpha), sigma = (T)a.sigma;
  // rounding bound of the check (FP32 iterations): |computed - FP64| <= kappa * sum |a_ij v_j|
  // per row, with the stored matrices and the outputs rounded to FP32 and FP64 accumulation over
  // at most L terms on both sides; an FP64 handle computes the FP64 residual itself
  const double kappa = sizeof(T) == sizeof(double) ? 0.0 : 1.01 * (2.0 * 0x1p-24 + 2.0 * (double)(L + 8) * 0x1p-53);
  const double ut = sizeof(T) == sizeof(double) ? 0.0 : 1.01 * 0x1p-24;
  // the state of row r, held by all S lanes of the row (they compute the same values); ax is
  // the last check's (A x)_r of a constraint row
  T sx = 0, sz = 0, sy = 0, sq = 0, sl = 0, su = 0;
  double ax = 0.0;
  int j = a.warm ? *a.js : a.j0;
  int held_j = -1;
  T wst[NI];  // this lane's entries of its row of the layer matrix, for penalty held_j

  for (int sv = 0; sv < a.count; ++sv) {
    const bool warm = sv == 0 ? a.warm != 0 : a.chain != 0;
    __syncthreads();  // upd[] of the previous solve has been read

    // update from an initial state (Sec. IV): q = F x0, l = lo - E x0, u = hi - E x0, FP64
    // products, one wave per row; written back to the handle's q, l, u
    if (a.x0) {
      const double* x0 = a.x0 + (long)sv * a.nx;
      for (int rr = wave; rr < L; rr += SWAVES) {
        const double* arow = rr < n ? a.F + (long)rr * a.nx : a.E + (long)(rr - n) * a.nx;
        double dv = 0.0;
        for (int c = lane; c < a.nx; c += kWave) dv = fma(arow[c], x0[c], dv);
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) dv += __shfl_xor(dv, off, kWave);
        if (lane == 0) {
          if (rr < n) {
            upd[rr][0] = (T)dv;
            static_cast<T*>(const_cast<void*>(a.q))[rr] = (T)dv;
          } else {
            const int i = rr - n;
            upd[rr][0] = (T)(a.plo[i] - dv);
            upd[rr][1] = (T)(a.phi[i] - dv);
            static_cast<T*>(const_cast<void*>(a.l))[i] = upd[rr][0];
            static_cast<T*>(const_cast<void*>(a.u))[i] = upd[rr][1];
          }
        }
      }
    }
    __syncthreads();

    // cold start (zero state, start penalty), or warm from the handle (first solve) or from the
    // previous solve of this launch
    if (row) {
      if (xrow) {
        sq = a.x0 ? upd[r][0] : static_cast<const T*>(a.q)[r];
        if (!warm) sx = (T)0;
        else if (sv == 0) sx = static_cast<const T*>(a.xs)[r];
      } else {
        const int i = r - n;
        sl = a.x0 ? upd[r][0] : static_cast<const T*>(a.l)[i];
        su = a.x0 ? upd[r][1] : static_cast<const T*>(a.u)[i];
        if (!warm) sy = (T)0;
        else if (sv == 0) sy = static_cast<const T*>(a.ys)[i];
        ax = 0.0;
        sz = (T)0;
      }
    }
    if (!warm) j = a.j0;
    T srho = (T)(grid_s[j] * (seq ? a.rho_eq_scale : 1.0));
    T rinv = (T)1 / srho;  // y / rho as y * (1 / rho): one rounding more, no division per iteration
    if (j != held_j) {
      load_row<T, S, NI>(a, j, row, r, s, wst);
      held_j = j;
    }

    // warm start (Sec. II-B): z = A x with FP64 accumulation
    if (warm) {
      if (own) cv[r] = xrow ? sx : sy;
      __syncthreads();
      double p, unused, unused2, unused3;
      check_products<T, S, NI>(a, Cl, s, n, cv, p, unused, unused2, unused3);  // rows past L hold zeros
      p = row_sum<S>(p);
      if (row && !xrow) {
        sz = (T)p;
        ax = p;
      }
    }
    if (own) wb[1][r] = xrow ? sigma * sx - sq : srho * sz - sy;
    __syncthreads();  // w_1

    int k = 0, nchk = 0;
    const long hoff = (long)sv * a.max_checks;
    while (true) {
      const int kend = (k / ci + 1) * ci < max_iter ? (k / ci + 1) * ci : max_iter;
      while (k < kend) {
        ++k;
        // layer matvec: row r of Wc_j times w_k, then the row-local update
        if (wave_rows) {
          const T* w = wb[k & 1];
          T acc = (T)0;
#pragma unroll
          for (int i0 = 0; i0 < NI; i0 += kBatch) {
            T xv[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) xv[b] = w[(i0 + b) * S + s];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) acc = fma(wst[i0 + b], xv[b], acc);
          }
          const T v = row_sum<S>(acc);
          if (row) {
          if (xrow) {
            sx = alpha * v + oma * sx;
          } else {
            const T t = alpha * v + oma * sz + sy * rinv;
            const T zn = box_clamp(t, sl, su);
            sy = srho * (t - zn);
            sz = zn;
          }
            if (own && k < kend) wb[(k + 1) & 1][r] = xrow ? sigma * sx - sq : srho * sz - sy;
          }
        }
        __syncthreads();
      }

      // check at iteration k: rows of [P, A'; A, 0] [x; y], FP64 accumulation: P x + A'y for
      // the x rows (dual side), A x for the constraint rows (primal side). In FP32 the published
      // residuals are upper bounds and the norms lower bounds of the FP64 values of a CPU
      // evaluation of the returned x, z, y with the caller's P, q, A (kappa), so SOLVED implies
      // that the FP64 test passes.
      if (own) cv[r] = xrow ? sx : sy;
      __syncthreads();
      double pr, ar, apr, aar;
      check_products<T, S, NI>(a, Cl, s, L, cv, pr, ar, apr, aar);
      pr = row_sum<S>(pr);
      ar = row_sum<S>(ar);
      apr = row_sum<S>(apr);
      aar = row_sum<S>(aar);
      if (row && !xrow) ax = pr;
      if (own) {
        // a Ruiz-scaled problem weights each row's terms so that the norms are the original
        // problem's: 1 / (c D_r) on the dual side, 1 / E_i on the primal side (1 otherwise)
        if (xrow) {
          const double qv = (double)sq, f = a.sc_dual ? a.sc_dual[r] : 1.0;
          const double dpx = kappa * apr, daty = kappa * aar, dq = ut * fabs(qv);
          nrm[K_RD][r] = abs_bits(f * (fabs(pr + qv + ar) + dpx + daty + dq));
          nrm[K_PX][r] = abs_bits(f * lower_bound(fabs(pr), dpx));
          nrm[K_ATY][r] = abs_bits(f * lower_bound(fabs(ar), daty));
          nrm[K_Q][r] = abs_bits(f * lower_bound(fabs(qv), dq));
          nrm[K_RP][r] = nrm[K_AX][r] = nrm[K_Z][r] = 0;
        } else {
          const double e = a.sc_prim ? a.sc_prim[r - n] : 1.0;
          const double ds = kappa * apr, zv = (double)sz, dz = ut * fabs(zv);
          nrm[K_RP][r] = abs_bits(e * (fabs(pr - zv) + ds + dz));
          nrm[K_AX][r] = abs_bits(e * lower_bound(fabs(pr), ds));
          nrm[K_Z][r] = abs_bits(e * lower_bound(fabs(zv), dz));
          nrm[K_RD][r] = nrm[K_PX][r] = nrm[K_ATY][r] = nrm[K_Q][r] = 0;
        }
      }
      __syncthreads();
      // wave w < 7 reduces norm w over the rows; wave 7 reads the host's abort flag
      if (wave < K_NORMS) {
        uint64_t m = 0;
        for (int rr = lane; rr < L; rr += kWave) m = nrm[wave][rr] > m ? nrm[wave][rr] : m;
        m = wave_max_u64(m);
        if (lane == 0) fin[wave] = m;
      } else if (wave == K_NORMS && lane == 0) {
        // the host-mapped flag costs a PCIe round trip, so it is read at every kAbortEvery-th
        // check only
        const bool ab = (nchk % kAbortEvery) == kAbortEvery - 1 && a.abort_flag &&
                        __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        fin[K_NORMS] = ab ? 1u : 0u;
      }
      __syncthreads();
      if (tid == 0) {
        bool nonfinite = false;
        for (int i = 0; i < K_NORMS; ++i) nonfinite |= fin[i] >= kInfBits;
        const double rp = bits_to_double(fin[K_RP]), rd = bits_to_double(fin[K_RD]);
        const double nax = bits_to_double(fin[K_AX]), nz = bits_to_double(fin[K_Z]);
        const double npx = bits_to_double(fin[K_PX]), naty = bits_to_double(fin[K_ATY]);
        const double nq = bits_to_double(fin[K_Q]);
        int st = S_RUNNING;
        if (nonfinite) {
          st = S_NONFINITE;
        } else if (a.terminate) {
          const double eps_p = a.eps_abs + a.eps_rel * fmax(nax, nz);
          const double eps_d = a.eps_abs + a.eps_rel * fmax(fmax(npx, naty), nq);
          if (rp <= eps_p && rd <= eps_d) st = S_SOLVED;
        }
        if (st == S_RUNNING && k == max_iter) st = S_MAX_ITER;
        if (st == S_RUNNING && fin[K_NORMS] == 1) st = S_ABORTED;
        int jn = j;
        if (st == S_RUNNING && a.n_rho > 1 && rp > 0.0 && rd > 0.0) {
          const double num = rp * fmax(fmax(npx, naty), fmax(nq, 1e-4));
          const double den = rd * fmax(fmax(nax, nz), 1e-4);
          const double rh = grid_s[j] * sqrt(num / den);
          jn = 0;
          while (jn < a.n_rho - 1 && rh > mid_s[jn]) ++jn;
        }
        if (a.rho_hist) a.rho_hist[hoff + nchk] = jn;
        if (a.prim_res) a.prim_res[hoff + nchk] = rp;
        if (a.dual_res) a.dual_res[hoff + nchk] = rd;
        decision[0] = st;
        decision[1] = jn;
      }
      __syncthreads();
      const int st = decision[0], jn = decision[1];
      ++nchk;
      if (st != S_RUNNING) {
        if (own) {
          // the handle keeps the (scaled) iterates; the outputs are in original units
          if (xrow) {
            static_cast<T*>(a.xs)[r] = sx;
            static_cast<T*>(a.xo)[(long)sv * n + r] = a.un_x ? (T)(a.un_x[r] * (double)sx) : sx;
          } else {
            const int i = r - n;
            static_cast<T*>(a.zs)[i] = sz;
            static_cast<T*>(a.ys)[i] = sy;
            a.axs[i] = ax;
            static_cast<T*>(a.zo)[(long)sv * a.m + i] = a.sc_prim ? (T)(a.sc_prim[i] * (double)sz) : sz;
            static_cast<T*>(a.yo)[(long)sv * a.m + i] = a.un_y ? (T)(a.un_y[i] * (double)sy) : sy;
          }
        }
        if (tid == 0) {
          a.iterations[sv] = k;
          a.status[sv] = st;
          a.rho_index[sv] = j;
          *a.js = j;
        }
        break;  // next solve of the sequence
      }
      if (jn != j) {
        j = jn;
        srho = (T)(grid_s[j] * (seq ? a.rho_eq_scale : 1.0));
        rinv = (T)1 / srho;
        load_row<T, S, NI>(a, j, row, r, s, wst);
        held_j = j;
      }
      if (own) wb[(k + 1) & 1][r] = xrow ? sigma * sx - sq : srho * sz - sy;
      __syncthreads();  // w_{k+1}; decision[] and fin[] are reused
    }
  }
}

template <typename T, int S, int NI>
const void* shape_fn() {
  return reinterpret_cast<const void*>(&small_kernel<T, S, NI>);
}
template <typename T, int S, int NI>
constexpr size_t shape_lds() {
  return (size_t)NI * SB * sizeof(T);  // the check matrix: at most 128 KB (FP64, NI = 16)
}

template <typename T, int S, int NI>
hipError_t prepare_shape() {
  return hipFuncSetAttribute(shape_fn<T, S, NI>(), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)shape_lds<T, S, NI>());
}

template <typename T, int S, int NI>
hipError_t launch_shape(const LayerArgs& a, hipStream_t st) {
  LayerArgs arg = a;
  void* args[] = {&arg};
  return hipLaunchKernel(shape_fn<T, S, NI>(), dim3(1), dim3(SB), args, shape_lds<T, S, NI>(), st);
}

}  // namespace

template <typename T>
hipError_t prepare_small(int L) {
  if (L < 1 || L > kSmallRows) return hipErrorInvalidValue;
  if (L <= 64) return prepare_shape<T, 8, 8>();
  if (L <= 96) return prepare_shape<T, 8, 12>();
  return prepare_shape<T, 8, 16>();
}

template <typename T>
hipError_t launch_small(const LayerArgs& a, hipStream_t st) {
  if (a.L < 1 || a.L > kSmallRows || a.Ad || a.n_rho > kRhoMax) return hipErrorInvalidValue;
  if (a.L <= 64) return launch_shape<T, 8, 8>(a, st);
  if (a.L <= 96) return launch_shape<T, 8, 12>(a, st);
  return launch_shape<T, 8, 16>(a, st);
}

template hipError_t prepare_small<float>(int);
template hipError_t prepare_small<double>(int);
template hipError_t launch_small<float>(const LayerArgs&, hipStream_t);
template hipError_t launch_small<double>(const LayerArgs&, hipStream_t);

}  // namespace rqp
