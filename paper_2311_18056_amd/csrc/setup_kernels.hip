// Offline-stage kernels in FP64 (Algorithm 1, "Offline"; D under eq. gpu_update).
//
// The layer needs D_j = (P + sigma I + A' diag(rho_j) A)^-1 for every grid penalty. It is formed
// here by an in-place blocked Gauss-Jordan inverse: for an SPD matrix every pivot block is a
// Schur complement of an SPD matrix, so no pivoting is needed, every step is a rank-32 update
// of the whole matrix (GEMM-shaped, no triangular solves), and a non-positive pivot is the
// positive-definiteness test the setup must report.
#include "setup_kernels.h"


namespace rqp {

namespace {

constexpr int GT = 64;  // GEMM output tile edge
constexpr int GK = 16;  // GEMM k-step
constexpr int SB = 32;  // Gauss-Jordan pivot block

__global__ void __launch_bounds__(256) gemm_f64_kernel(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                       long a_rs, long a_cs, const double* __restrict__ ks,
                                                       const double* __restrict__ B, long b_rs, long b_cs, double beta,
                                                       double* __restrict__ C, long ldc) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  const bool a_kfast = a_cs == 1;  // consecutive k contiguous in memory
  const bool b_jfast = b_cs == 1;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;

  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int e = tid; e < GT * GK; e += 256) {
      int r, kk;
      if (a_kfast) {
        r = e / GK;
        kk = e % GK;
      } else {
        kk = e / GT;
        r = e % GT;
      }
      int gi = i0 + r, gk = k0 + kk;
      double v = 0.0;
      if (gi < M && gk < K) {
        v = A[(long)gi * a_rs + (long)gk * a_cs];
        if (ks) v *= ks[gk];
      }
      As[kk][r] = v;
      int c;
      if (b_jfast) {
        kk = e / GT;
        c = e % GT;
      } else {
        c = e / GK;
        kk = e % GK;
      }
      int gj = j0 + c;
      gk = k0 + kk;
      Bs[kk][c] = (gj < N && gk < K) ? B[(long)gk * b_rs + (long)gj * b_cs] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int gi = i0 + ty + 16 * a;
    if (gi >= M) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int gj = j0 + tx + 16 * b;
      if (gj >= N) continue;
      double* c = C + (long)gi * ldc + gj;
      *c = (beta == 0.0) ? alpha * acc[a][b] : alpha * acc[a][b] + beta * (*c);
    }
  }
}

__global__ void kkt_form_kernel(int n, const double* __restrict__ P, const double* __restrict__ Gw, double sigma,
                                double rho, double* __restrict__ K) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)n * n;
  if (idx >= total) return;
  int i = (int)(idx / n), j = (int)(idx % n);
  double v = P[idx] + rho * Gw[idx];
  if (i == j) v += sigma;
  K[idx] = v;
}

// Inverse of the pivot block (bb x bb, bb <= 32) by unblocked Gauss-Jordan in LDS.
__global__ void __launch_bounds__(1024) gj_diag_kernel(const double* __restrict__ M, int n, int pb, int bb,
                                                       double* __restrict__ Pinv, int* __restrict__ info) {
  __shared__ double S[SB][SB + 1];
  const int r = threadIdx.x / SB, c = threadIdx.x % SB;
  const bool act = r < bb && c < bb;
  S[r][c] = act ? M[(long)(pb + r) * n + pb + c] : 0.0;
  __syncthreads();
  for (int k = 0; k < bb; ++k) {
    double piv = S[k][k];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) *info = 1;
      piv = 1.0;  // keep the arithmetic finite; the caller reports the failure
    }
    double srk = S[r][k], skc = S[k][c], src = S[r][c];
    __syncthreads();
    double v;
    if (r == k && c == k)
      v = 1.0 / piv;
    else if (r == k)
      v = skc / piv;
    else if (c == k)
      v = -srk / piv;
    else
      v = src - srk * (skc / piv);
    if (act) S[r][c] = v;
    __syncthreads();
  }
  Pinv[r * SB + c] = act ? S[r][c] : 0.0;
}

// Row panel R = Pinv * M[pb:pb+bb, :] (bb x n) and a copy of the old column panel
// Cold = M[:, pb:pb+bb] (n x 32), both from the matrix before this step.
__global__ void __launch_bounds__(256) gj_panel_kernel(const double* __restrict__ M, int n, int pb, int bb,
                                                       const double* __restrict__ Pinv, double* __restrict__ R,
                                                       double* __restrict__ Cold) {
  __shared__ double Ps[SB][SB + 1];
  __shared__ double Ms[SB][GT + 1];
  const int tid = threadIdx.x;
  const int j0 = blockIdx.x * GT;
  for (int e = tid; e < SB * SB; e += 256) Ps[e / SB][e % SB] = Pinv[e];
  for (int e = tid; e < SB * GT; e += 256) {
    int t = e / GT, c = e % GT;
    int gj = j0 + c;
    Ms[t][c] = (t < bb && gj < n) ? M[(long)(pb + t) * n + gj] : 0.0;
  }
  // old column panel rows j0..j0+63 (M is symmetric in exact arithmetic, but keep the column)
  for (int e = tid; e < GT * SB; e += 256) {
    int r = e / SB, t = e % SB;
    int gi = j0 + r;
    if (gi < n) Cold[(long)gi * SB + t] = (t < bb) ? M[(long)gi * n + pb + t] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < SB * GT; e += 256) {
    int t = e / GT, c = e % GT;
    int gj = j0 + c;
    if (t >= bb || gj >= n) continue;
    double s = 0.0;
    for (int k = 0; k < bb; ++k) s = fma(Ps[t][k], Ms[k][c], s);
    R[(long)t * n + gj] = s;
  }
}

// Trailing update of one Gauss-Jordan step on a 64 x 64 tile of M.
__global__ void __launch_bounds__(256) gj_update_kernel(double* __restrict__ M, int n, int pb, int bb,
                                                        const double* __restrict__ Pinv, const double* __restrict__ R,
                                                        const double* __restrict__ Cold) {
  __shared__ double Cs[SB][GT + 1];  // Cs[t][i] = Cold[i0 + i][t]
  __shared__ double Rs[SB][GT + 1];  // Rs[t][j] = R[t][j0 + j]
  __shared__ double Ps[SB][SB + 1];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  for (int e = tid; e < SB * SB; e += 256) Ps[e / SB][e % SB] = Pinv[e];
  for (int e = tid; e < GT * SB; e += 256) {
    int i = e / SB, t = e % SB;
    int gi = i0 + i;
    Cs[t][i] = (gi < n) ? Cold[(long)gi * SB + t] : 0.0;
  }
  for (int e = tid; e < SB * GT; e += 256) {
    int t = e / GT, j = e % GT;
    int gj = j0 + j;
    Rs[t][j] = (t < bb && gj < n) ? R[(long)t * n + gj] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int ii = ty + 16 * a;
    int gi = i0 + ii;
    if (gi >= n) continue;
    bool in_i = gi >= pb && gi < pb + bb;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int jj = tx + 16 * b;
      int gj = j0 + jj;
      if (gj >= n) continue;
      bool in_j = gj >= pb && gj < pb + bb;
      double* mp = M + (long)gi * n + gj;
      if (in_i && in_j) {
        *mp = Ps[gi - pb][gj - pb];
      } else if (in_i) {
        *mp = Rs[gi - pb][jj];
      } else if (in_j) {
        double s = 0.0;
        for (int t = 0; t < bb; ++t) s = fma(Cs[t][ii], Ps[t][gj - pb], s);
        *mp = -s;
      } else {
        double s = 0.0;
        for (int t = 0; t < bb; ++t) s = fma(Cs[t][ii], Rs[t][jj], s);
        *mp -= s;
      }
    }
  }
}

__global__ void symmetrize_kernel(int n, double* __restrict__ M) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * n) return;
  int i = (int)(idx / n), j = (int)(idx % n);
  if (i >= j) return;
  double a = M[(long)i * n + j], b = M[(long)j * n + i];
  double v = 0.5 * (a + b);
  M[(long)i * n + j] = v;
  M[(long)j * n + i] = v;
}

template <typename T>
__global__ void assemble_layer_kernel(int n, int m, const double* __restrict__ D, const double* __restrict__ DAt,
                                      const double* __restrict__ ADAt, T* __restrict__ W, long ldw) {
  const int L = n + m;
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)L * ldw) return;
  int i = (int)(idx / ldw), j = (int)(idx % ldw);
  double v = 0.0;
  if (j < L) {
    if (i < n && j < n)
      v = D[(long)i * n + j];
    else if (i < n)
      v = DAt[(long)i * m + (j - n)];
    else if (j < n)
      v = DAt[(long)j * m + (i - n)];
    else
      v = ADAt[(long)(i - n) * m + (j - n)];
  }
  W[idx] = (T)v;
}

template <typename T>
__global__ void assemble_check_kernel(int n, int m, const double* __restrict__ P, const double* __restrict__ A,
                                      T* __restrict__ C, long ldw) {
  const int L = n + m;
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)L * ldw) return;
  int i = (int)(idx / ldw), j = (int)(idx % ldw);
  double v = 0.0;
  if (j < L) {
    if (i < n && j < n)
      v = P[(long)i * n + j];
    else if (i < n)
      v = A[(long)(j - n) * n + i];
    else if (j < n)
      v = A[(long)(i - n) * n + j];
  }
  C[idx] = (T)v;
}

template <typename T>
__global__ void cast_kernel(long count, const double* __restrict__ x, const double* __restrict__ f, long period,
                            T* __restrict__ y) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) y[idx] = f ? (T)(x[idx] * f[idx % period]) : (T)x[idx];
}

// One wave per output row: q rows first, then the m constraint rows. Writes the vectors
// straight in the iteration precision T.
template <typename T>
__global__ void __launch_bounds__(256) mpc_vectors_kernel(long B, int n, int m, int nx, const double* __restrict__ F,
                                                          const double* __restrict__ E, const double* __restrict__ lo,
                                                          const double* __restrict__ hi,
                                                          const double* __restrict__ x0, T* __restrict__ q,
                                                          T* __restrict__ l, T* __restrict__ u) {
  const long grow = (long)blockIdx.x * 4 + threadIdx.x / 64;  // instance * (n + m) + row
  const int lane = threadIdx.x % 64;
  if (grow >= B * (n + m)) return;
  const long b = grow / (n + m);
  const int row = (int)(grow % (n + m));
  const double* a = row < n ? F + (long)row * nx : E + (long)(row - n) * nx;
  const double* xb = x0 + b * nx;
  double s = 0.0;
  for (int c = lane; c < nx; c += 64) s = fma(a[c], xb[c], s);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) {
    if (row < n) {
      q[b * n + row] = (T)s;
    } else {
      const int i = row - n;
      l[b * m + i] = (T)(lo[i] - s);
      u[b * m + i] = (T)(hi[i] - s);
    }
  }
}

// Many instances at once: the same vectors as a tiled FP64 product [F; E] X0' (64 rows x 64
// instances per block, nx in chunks of 32 through LDS); every output is one FMA chain over
// k = 0 .. nx-1 in order, the order a thread-per-output loop gives too.
constexpr int MT = 64, MK = 32;
template <typename T>
__global__ void __launch_bounds__(256) mpc_tiled_kernel(int B, int n, int m, int nx, const double* __restrict__ F,
                                                        const double* __restrict__ E, const double* __restrict__ lo,
                                                        const double* __restrict__ hi, const double* __restrict__ x0,
                                                        T* __restrict__ q, T* __restrict__ l, T* __restrict__ u) {
  __shared__ double fe[MT][MK + 1];
  __shared__ double xs[MT][MK + 1];
  const int L = n + m, r0 = blockIdx.x * MT, b0 = blockIdx.y * MT, tid = threadIdx.x;
  const int tr = tid % 16, tb = tid / 16;  // rows tr + 16 i, instances tb + 16 j
  double acc[4][4] = {};
  for (int k0 = 0; k0 < nx; k0 += MK) {
    for (int e = tid; e < MT * MK; e += 256) {
      const int rr = e / MK, kk = e % MK, R = r0 + rr, b = b0 + rr, k = k0 + kk;
      fe[rr][kk] = (R < L && k < nx) ? (R < n ? F[(long)R * nx + k] : E[(long)(R - n) * nx + k]) : 0.0;
      xs[rr][kk] = (b < B && k < nx) ? x0[(long)b * nx + k] : 0.0;
    }
    __syncthreads();
    const int kn = min(MK, nx - k0);
    for (int kk = 0; kk < kn; ++kk)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(fe[tr + 16 * i][kk], xs[tb + 16 * j][kk], acc[i][j]);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int R = r0 + tr + 16 * i, b = b0 + tb + 16 * j;
      if (R >= L || b >= B) continue;
      if (R < n) {
        q[(long)b * n + R] = (T)acc[i][j];
      } else {
        const int ii = R - n;
        l[(long)b * m + ii] = (T)(lo[ii] - acc[i][j]);
        u[(long)b * m + ii] = (T)(hi[ii] - acc[i][j]);
      }
    }
}

inline unsigned blocks_for(long count, int bs) { return (unsigned)((count + bs - 1) / bs); }

}  // namespace

hipError_t gemm_f64(int M, int N, int K, double alpha, const double* A, long a_rs, long a_cs, const double* kscale,
                    const double* B, long b_rs, long b_cs, double beta, double* C, long ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, st, M, N, K, alpha, A, a_rs, a_cs, kscale, B, b_rs, b_cs,
                     beta, C, ldc);
  return hipGetLastError();
}

hipError_t kkt_form_f64(int n, const double* P, const double* Gw, double sigma, double rho, double* K, hipStream_t st) {
  long total = (long)n * n;
  hipLaunchKernelGGL(kkt_form_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st, n, P, Gw, sigma, rho, K);
  return hipGetLastError();
}

hipError_t spd_inverse_f64(int n, double* M, double* work, int* info, hipStream_t st) {
  double* Pinv = work;
  double* R = work + SB * SB;
  double* Cold = R + (long)SB * n;
  const unsigned ct = (n + GT - 1) / GT;
  for (int pb = 0; pb < n; pb += SB) {
    int bb = n - pb < SB ? n - pb : SB;
    hipLaunchKernelGGL(gj_diag_kernel, dim3(1), dim3(SB * SB), 0, st, M, n, pb, bb, Pinv, info);
    hipLaunchKernelGGL(gj_panel_kernel, dim3(ct), dim3(256), 0, st, M, n, pb, bb, Pinv, R, Cold);
    hipLaunchKernelGGL(gj_update_kernel, dim3(ct, ct), dim3(256), 0, st, M, n, pb, bb, Pinv, R, Cold);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  long total = (long)n * n;
  hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st, n, M);
  return hipGetLastError();
}

template <typename T>
hipError_t assemble_layer(int n, int m, const double* D, const double* DAt, const double* ADAt, T* W, long ldw,
                          hipStream_t st) {
  long total = (long)(n + m) * ldw;
  hipLaunchKernelGGL(assemble_layer_kernel<T>, dim3(blocks_for(total, 256)), dim3(256), 0, st, n, m, D, DAt, ADAt, W,
                     ldw);
  return hipGetLastError();
}

template <typename T>
hipError_t assemble_check(int n, int m, const double* P, const double* A, T* C, long ldw, hipStream_t st) {
  long total = (long)(n + m) * ldw;
  hipLaunchKernelGGL(assemble_check_kernel<T>, dim3(blocks_for(total, 256)), dim3(256), 0, st, n, m, P, A, C, ldw);
  return hipGetLastError();
}

template <typename T>
hipError_t mpc_vectors(int B, int n, int m, int nx, const double* F, const double* E, const double* lo,
                       const double* hi, const double* x0, T* q, T* l, T* u, hipStream_t st) {
  const long rows = (long)B * (n + m);
  hipLaunchKernelGGL(mpc_vectors_kernel<T>, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, (long)B, n, m, nx, F, E,
                     lo, hi, x0, q, l, u);
  return hipGetLastError();
}

template <typename T>
hipError_t mpc_vectors_tiled(int B, int n, int m, int nx, const double* F, const double* E, const double* lo,
                             const double* hi, const double* x0, T* q, T* l, T* u, hipStream_t st) {
  const dim3 grid((unsigned)((n + m + MT - 1) / MT), (unsigned)((B + MT - 1) / MT));
  hipLaunchKernelGGL(mpc_tiled_kernel<T>, grid, dim3(256), 0, st, B, n, m, nx, F, E, lo, hi, x0, q, l, u);
  return hipGetLastError();
}

template <typename T>
hipError_t cast_from_f64(long count, const double* x, T* y, hipStream_t st, const double* f, long period) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(cast_kernel<T>, dim3(blocks_for(count, 256)), dim3(256), 0, st, count, x, f,
                     period > 0 ? period : 1, y);
  return hipGetLastError();
}

template hipError_t assemble_layer<float>(int, int, const double*, const double*, const double*, float*, long,
                                          hipStream_t);
template hipError_t assemble_layer<double>(int, int, const double*, const double*, const double*, double*, long,
                                           hipStream_t);
template hipError_t assemble_check<float>(int, int, const double*, const double*, float*, long, hipStream_t);
template hipError_t assemble_check<double>(int, int, const double*, const double*, double*, long, hipStream_t);
template hipError_t mpc_vectors<float>(int, int, int, int, const double*, const double*, const double*,
                                       const double*, const double*, float*, float*, float*, hipStream_t);
template hipError_t mpc_vectors<double>(int, int, int, int, const double*, const double*, const double*,
                                        const double*, const double*, double*, double*, double*, hipStream_t);
template hipError_t mpc_vectors_tiled<float>(int, int, int, int, const double*, const double*, const double*,
                                             const double*, const double*, float*, float*, float*, hipStream_t);
template hipError_t cast_from_f64<float>(long, const double*, float*, hipStream_t, const double*, long);
template hipError_t cast_from_f64<double>(long, const double*, double*, hipStream_t, const double*, long);

}  // namespace rqp
