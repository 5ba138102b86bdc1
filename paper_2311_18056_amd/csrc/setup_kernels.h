// Offline-stage kernels (Algorithm 1, "Offline"): FP64 products and the KKT inverse on the GPU.
#pragma once
#include <hip/hip_runtime.h>

namespace rqp {

// C = alpha * op(A) op(B) + beta * C for an M x N result, where
//   op(A)(i, k) = A[i * a_rs + k * a_cs] * (kscale ? kscale[k] : 1),  op(B)(k, j) = B[k * b_rs + j * b_cs],
// and C is row-major with leading dimension ldc. Any strides, so transposes are free.
hipError_t gemm_f64(int M, int N, int K, double alpha, const double* A, long a_rs, long a_cs, const double* kscale,
                    const double* B, long b_rs, long b_cs, double beta, double* C, long ldc, hipStream_t st);

// K = P + sigma I + rho * Gw  (all n x n, row-major, leading dimension n).
hipError_t kkt_form_f64(int n, const double* P, const double* Gw, double sigma, double rho, double* K, hipStream_t st);

// In-place inverse of a symmetric positive definite n x n matrix by blocked Gauss-Jordan
// elimination without pivoting (every pivot block is a Schur complement of an SPD matrix, so
// no pivoting is needed and a non-positive pivot proves the matrix is not positive definite).
// work must hold 2*32*n + 32*32 doubles. *info (device int) is set to 1 on a bad pivot; the
// caller zeroes it first. The result is symmetrised.
hipError_t spd_inverse_f64(int n, double* M, double* work, int* info, hipStream_t st);

// Layer weights of the compact form: rows/cols [0, n) x [0, n) = D, [0, n) x [n, L) = D A',
// [n, L) x [0, n) = (D A')', [n, L) x [n, L) = A D A'; written as T with leading dimension ldw.
template <typename T>
hipError_t assemble_layer(int n, int m, const double* D, const double* DAt, const double* ADAt, T* W, long ldw,
                          hipStream_t st);

// Check matrix [P, A'; A, 0] as T with leading dimension ldw (residual products).
template <typename T>
hipError_t assemble_check(int n, int m, const double* P, const double* A, T* C, long ldw, hipStream_t st);

// Parametric QP vectors of condensed MPC (Sec. IV) for B instances: q_b = F x0_b,
// l_b = lo - E x0_b, u_b = hi - E x0_b; F n x nx and E m x nx row-major FP64 on the device,
// x0 B x nx; accumulated in FP64 and written as T (q: B x n, l and u: B x m).
template <typename T>
hipError_t mpc_vectors(int B, int n, int m, int nx, const double* F, const double* E, const double* lo,
                       const double* hi, const double* x0, T* q, T* l, T* u, hipStream_t st);
// The same for many instances as a tiled FP64 product; each output is one in-order FMA chain
// over the nx entries of x0 (the batched engine and its slot loader use this order).
template <typename T>
hipError_t mpc_vectors_tiled(int B, int n, int m, int nx, const double* F, const double* E, const double* lo,
                             const double* hi, const double* x0, T* q, T* l, T* u, hipStream_t st);

// y = x cast to T (count elements); with f: y[i] = x[i] * f[i % period] cast to T.
template <typename T>
hipError_t cast_from_f64(long count, const double* x, T* y, hipStream_t st, const double* f = nullptr,
                         long period = 1);

}  // namespace rqp
