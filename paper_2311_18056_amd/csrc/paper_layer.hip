// The paper's literal weight-tied layer (eq. gpu_update) on the GPU, for comparison with the
// compact form: see paper_layer.h.
#include "paper_layer.h"

#include "device_common.h"
#include "setup_kernels.h"

namespace rqp {
namespace {

constexpr int BS = kPaperBlock;
constexpr int NWAVE = BS / kWave;
constexpr unsigned kSpinLimit = 1u << 22;

int blocks_for(long count, int bs) { return (int)((count + bs - 1) / bs); }

template <typename T>
__global__ void to_f64_kernel(int rows, int cols, const T* __restrict__ src, long ld, double* __restrict__ dst) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  const int i = (int)(idx / cols), j = (int)(idx % cols);
  dst[idx] = (double)src[(long)i * ld + j];
}

// Entry (i, j) of W, block by block as eq. gpu_update writes it (R = diag(rho)):
//   x rows:      D (sigma I - A'RA),          2 D A' R,         -D A'
//   z rows:      A D (sigma I - A'RA) + A,    2 A D A' R - I,   -A D A' + R^-1
//   dual rows:   R A,                         -R,               I
// with Wc the FP64 compact matrix [D, D A'; A D, A D A'] (L x L), A (m x n),
// T1 = (D A') R A (n x n) and T2 = (A D A') R A (m x n).
template <typename T>
__global__ void paper_w_kernel(int n, int m, const double* __restrict__ Wc, const double* __restrict__ A,
                               const double* __restrict__ T1, const double* __restrict__ T2,
                               const double* __restrict__ rho, double sigma, T* __restrict__ W, long ldp) {
  const int L = n + m, Lp = n + 2 * m;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)Lp * ldp) return;
  const int i = (int)(idx / ldp), j = (int)(idx % ldp);
  double v = 0.0;
  if (j < Lp) {
    if (i < n) {
      if (j < n)
        v = sigma * Wc[(long)i * L + j] - T1[(long)i * n + j];
      else if (j < n + m)
        v = 2.0 * Wc[(long)i * L + j] * rho[j - n];
      else
        v = -Wc[(long)i * L + (j - m)];
    } else if (i < n + m) {
      const int ii = i - n;
      if (j < n)
        v = sigma * Wc[(long)i * L + j] - T2[(long)ii * n + j] + A[(long)ii * n + j];
      else if (j < n + m)
        v = 2.0 * Wc[(long)i * L + j] * rho[j - n] - (j - n == ii ? 1.0 : 0.0);
      else
        v = -Wc[(long)i * L + (j - m)] + (j - n - m == ii ? 1.0 / rho[ii] : 0.0);
    } else {
      const int ii = i - n - m;
      if (j < n)
        v = rho[ii] * A[(long)ii * n + j];
      else if (j < n + m)
        v = (j - n == ii) ? -rho[ii] : 0.0;
      else
        v = (j - n - m == ii) ? 1.0 : 0.0;
    }
  }
  W[idx] = (T)v;
}

__device__ __forceinline__ bool err_set(const unsigned* err, uint32_t tag) {
  return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == tag;
}

// 16-byte vectors of T for the row products
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float __attribute__((ext_vector_type(4))) type;
  static constexpr int kLen = 4;
};
template <>
struct Vec16<double> {
  typedef double __attribute__((ext_vector_type(2))) type;
  static constexpr int kLen = 2;
};

// One workgroup owns a contiguous block of rows of W. Per layer: every thread polls its share of
// the previous v into LDS, then each wave forms two owned rows at a time, (W v)_row + b_row
// (16-byte loads of both rows, lane-strided products in T, butterfly sums), clamps z rows to
// [l, u] and publishes the entries with the next tag. The weights are read from memory every
// layer. W rows and the LDS copy of v are zero-padded to ldp (a multiple of 4).
template <typename T>
__global__ void __launch_bounds__(BS) paper_layer_kernel(PaperArgs a) {
  constexpr int NW = LLWords<T>::kWords;
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  T* vsh = reinterpret_cast<T*>(dyn_lds);  // the layer input, ldp entries (zeros past Lp)
  __shared__ T own[kPaperMaxRows], bsh[kPaperMaxRows], lo[kPaperMaxRows], hi[kPaperMaxRows];
  __shared__ int fail;
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid % kWave, wave = tid / kWave;
  const int n = a.n, m = a.m, Lp = a.Lp;
  const int rbase = Lp / G, rextra = Lp % G;
  const int nrows = rbase + (g < rextra ? 1 : 0);
  const int r0 = g * rbase + (g < rextra ? g : rextra);
  const T* q = static_cast<const T*>(a.q);
  if (tid == 0) fail = 0;
  for (int c = Lp + tid; c < a.ldp; c += BS) vsh[c] = (T)0;
  // b = -[D; A D] q (x and z rows; the compact matrix's first n columns), 0 for the dual rows
  for (int rr = wave; rr < nrows; rr += NWAVE) {
    const int R = r0 + rr;
    double dv = 0.0;
    if (R < n + m) {
      const T* row = static_cast<const T*>(a.Wc) + (long)R * a.ldw;
      for (int c = lane; c < n; c += kWave) dv = fma((double)row[c], (double)q[c], dv);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) dv += __shfl_xor(dv, off, kWave);
    if (lane == 0) {
      const bool zr = R >= n && R < n + m;
      bsh[rr] = (T)(-dv);
      lo[rr] = zr ? static_cast<const T*>(a.l)[R - n] : (T)0;
      hi[rr] = zr ? static_cast<const T*>(a.u)[R - n] : (T)0;
      own[rr] = (T)0;
    }
  }
  __syncthreads();
  const uint32_t tag = a.tag;
  // v_0 = 0, read by layer 1 from parity 1
  if (tid < nrows) ll_store(a.xw + ((long)Lp + r0 + tid) * NW, (T)0, tag + 1u);
  for (int k = 1; k <= a.iters; ++k) {
    const uint32_t want = tag + (uint32_t)k;
    const uint64_t* buf = a.xw + (long)(k & 1) * Lp * NW;
    bool bad = false;
    for (int c = tid; c < Lp && !bad; c += BS) {
      const uint64_t* p = buf + (long)c * NW;
      uint64_t w0 = ll_load_word(p), w1 = NW == 2 ? ll_load_word(p + 1) : ((uint64_t)want << 32);
      unsigned spins = 0;
      while (ll_tag(w0) != want || ll_tag(w1) != want) {
        w0 = ll_load_word(p);
        if (NW == 2) w1 = ll_load_word(p + 1);
        if ((++spins & 255u) == 0u && (spins > kSpinLimit || err_set(a.err, tag))) {
          bad = true;
          fail = 1;
          break;
        }
      }
      if constexpr (NW == 1)
        vsh[c] = ll_value_f(w0);
      else
        vsh[c] = bits_to_double(ll_bits64(w0, w1));
    }
    __syncthreads();
    if (fail) {
      if (tid == 0) __hip_atomic_store(a.err, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (g == 0 && tid == 0) {
        *a.iterations = k - 1;
        *a.status = 5;  // internal error
      }
      return;
    }
    typedef typename Vec16<T>::type V;
    constexpr int E = Vec16<T>::kLen;
    const int nvec = (int)(a.ldp / E);
    const V* vv = reinterpret_cast<const V*>(vsh);
    for (int rb = 2 * wave; rb < nrows; rb += 2 * NWAVE) {
      // rows rb and rb + 1 (the second clamped to a valid row; its result is not used)
      const int rr1 = rb + 1 < nrows ? rb + 1 : rb;
      const V* w0 = reinterpret_cast<const V*>(static_cast<const T*>(a.W) + (long)(r0 + rb) * a.ldp);
      const V* w1 = reinterpret_cast<const V*>(static_cast<const T*>(a.W) + (long)(r0 + rr1) * a.ldp);
      T acc0 = (T)0, acc1 = (T)0;
#pragma unroll 4
      for (int c = lane; c < nvec; c += kWave) {
        const V x = vv[c], p0 = w0[c], p1 = w1[c];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          acc0 = fma(p0[e], x[e], acc0);
          acc1 = fma(p1[e], x[e], acc1);
        }
      }
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) {
        acc0 += __shfl_xor(acc0, off, kWave);
        acc1 += __shfl_xor(acc1, off, kWave);
      }
      if (lane == 0) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int rr = rb + t;
          if (rr >= nrows) break;
          const int R = r0 + rr;
          T s = (t == 0 ? acc0 : acc1) + bsh[rr];
          if (R >= n && R < n + m) s = s < lo[rr] ? lo[rr] : (s > hi[rr] ? hi[rr] : s);
          own[rr] = s;
          if (k < a.iters) ll_store(a.xw + ((long)((k + 1) & 1) * Lp + R) * NW, s, tag + (uint32_t)(k + 1));
        }
      }
    }
    __syncthreads();  // vsh is overwritten by the next gather
  }
  if (tid < nrows) {
    const int R = r0 + tid;
    if (R < n)
      static_cast<T*>(a.xo)[R] = own[tid];
    else if (R < n + m)
      static_cast<T*>(a.zo)[R - n] = own[tid];
    else
      static_cast<T*>(a.yo)[R - n - m] = own[tid];
  }
  if (g == 0 && tid == 0) {
    *a.iterations = a.iters;
    *a.status = 2;  // the fixed count ran out
  }
}

}  // namespace

template <typename T>
hipError_t assemble_paper_w(int n, int m, const T* Wc, long ldw, const T* C, const double* rho, double sigma, T* W,
                            long ldp, hipStream_t st) {
  const int L = n + m, Lp = n + 2 * m;
  double *Wc64 = nullptr, *A64 = nullptr, *T1 = nullptr, *T2 = nullptr;
  hipError_t e = hipMalloc(&Wc64, (size_t)L * L * 8);
  if (e == hipSuccess) e = hipMalloc(&A64, (size_t)m * n * 8);
  if (e == hipSuccess) e = hipMalloc(&T1, (size_t)n * n * 8);
  if (e == hipSuccess) e = hipMalloc(&T2, (size_t)m * n * 8);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(to_f64_kernel<T>, dim3(blocks_for((long)L * L, 256)), dim3(256), 0, st, L, L, Wc, ldw, Wc64);
    hipLaunchKernelGGL(to_f64_kernel<T>, dim3(blocks_for((long)m * n, 256)), dim3(256), 0, st, m, n,
                       C + (long)n * ldw, ldw, A64);
    e = hipGetLastError();
  }
  // T1 = (D A') R A, T2 = (A D A') R A
  if (e == hipSuccess) e = gemm_f64(n, n, m, 1.0, Wc64 + n, L, 1, rho, A64, n, 1, 0.0, T1, n, st);
  if (e == hipSuccess) e = gemm_f64(m, n, m, 1.0, Wc64 + (long)n * L + n, L, 1, rho, A64, n, 1, 0.0, T2, n, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(paper_w_kernel<T>, dim3(blocks_for((long)Lp * ldp, 256)), dim3(256), 0, st, n, m, Wc64, A64, T1,
                       T2, rho, sigma, W, ldp);
    e = hipGetLastError();
  }
  const hipError_t es = hipStreamSynchronize(st);
  if (e == hipSuccess) e = es;
  for (double* p : {Wc64, A64, T1, T2})
    if (p) (void)hipFree(p);
  return e;
}

template <typename T>
hipError_t launch_paper_layer(const PaperArgs& a, int grid, hipStream_t st) {
  const size_t dyn = (size_t)a.ldp * sizeof(T);
  const void* fn = reinterpret_cast<const void*>(&paper_layer_kernel<T>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
  if (e != hipSuccess) return e;
  PaperArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(BS), args, dyn, st);
}

template hipError_t assemble_paper_w<float>(int, int, const float*, long, const float*, const double*, double, float*,
                                            long, hipStream_t);
template hipError_t assemble_paper_w<double>(int, int, const double*, long, const double*, const double*, double,
                                             double*, long, hipStream_t);
template hipError_t launch_paper_layer<float>(const PaperArgs&, int, hipStream_t);
template hipError_t launch_paper_layer<double>(const PaperArgs&, int, hipStream_t);

}  // namespace rqp
