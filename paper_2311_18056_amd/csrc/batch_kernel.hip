// Batched persistent ReLU-QP solve on the matrix cores (gfx950).
//
// B instances share P and A, hence the layer matrices Wc_j = [D_j, D_jA'; AD_j, AD_jA'] of the
// penalty grid; each has its own q, l, u, state (x, z, y), penalty index j_b and termination.
// One iteration for all active instances is the GEMM  OUT[b][r] = sum_c V[b][c] Wc_{j_b}[r][c]
// with V[b] = [sigma x_b - q_b ; rho_b z_b - y_b], followed by the row-local update of the
// single-instance kernel (relaxation, clamp, dual update) fused into the GEMM epilogue, which
// also writes the next V. Instances are grouped by penalty index so that a tile of 128
// instances uses one matrix; tiles are 128 instances x 128 layer rows, K in steps of 32.
//
// Precision: FP32 operands on v_mfma_f32_32x32x2_f32, or BF16 high/low splits of both operands
// with three products hi*hi + lo*hi + hi*lo on v_mfma_f32_32x32x16_bf16 (FP32 accumulation),
// which keeps ~16 significant bits of each operand; iterates stay FP32.
//
// Every check_interval iterations a GEMM in FP64 with the check matrix [P, A'; A, 0] (the FP64
// problem data) and the operand [x; y] (exact FP64 copies of the FP32 iterates) gives P x, A'y
// and A x of every instance on the FP64 matrix cores, so the residuals of eqs. primal and dual
// are FP64 evaluations of the state the solve returns; per-instance inf-norms are reduced with
// integer max on ordered FP64 bit patterns (atomics across row tiles), then one thread per
// instance applies the stopping test and the penalty rule. Phases are separated by a grid
// barrier (cooperative launch). An instance's arithmetic never depends on which other
// instances share its tiles, so a result is the same alone and in a batch.
#include "batch_kernel.h"

#include "device_common.h"

namespace rqp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));

constexpr int BS = kBatchBlock;
constexpr int TM = kTileM, TN = kTileN, TK = kTileK;
constexpr int PADB = 8;  // bf16 row padding in LDS (elements)
constexpr int PADF = 4;  // fp32 row padding in LDS (elements)
constexpr unsigned kBarSpin = 1u << 24;

enum { ST_RUNNING = 0, ST_SOLVED = 1, ST_MAX_ITER = 2, ST_NONFINITE = 3, ST_ABORTED = 4, ST_INTERNAL = 5 };
enum { N_RP = 0, N_RD, N_AX, N_Z, N_PX, N_ATY, N_Q };

__device__ __forceinline__ unsigned ld_acq(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Two-level grid barrier (8 groups by blockIdx % 8, then a global counter and a flag word).
// Counters are monotone: barrier number e completes when they reach e * size. Returns false
// if a wait exceeded the spin bound or another workgroup gave up (bar[1] set); every
// workgroup then leaves the kernel.
__device__ bool grid_barrier(unsigned* bar, unsigned e) {
  __shared__ int ok_s;
  // every wave's stores are made visible at device scope before its workgroup arrives
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned G = gridDim.x, g = blockIdx.x & 7u, ng = G < 8 ? G : 8;
    const unsigned gsize = (G - g + 7u) / 8u;
    int ok = 1;
    const unsigned old = __hip_atomic_fetch_add(bar + 64 + 32 * g, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (old == e * gsize - 1u) {
      const unsigned o2 = __hip_atomic_fetch_add(bar + 32, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (o2 == e * ng - 1u) __hip_atomic_store(bar, e, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned spins = 0;
    while (ld_acq(bar) < e) {
      if (++spins > kBarSpin || ld_acq(bar + 1) != 0u) {
        ok = 0;
        __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    ok_s = ok;
  }
  __syncthreads();
  return ok_s != 0;
}

// BF16 round to nearest even; the low part takes the rounding error, so hi + lo carries ~16
// significant bits.
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// Element (row, c) of a K-blocked operand with `rows` padded rows.
__device__ __forceinline__ long opidx(long rows, long row, int c) { return ((long)(c / TK) * rows + row) * TK + (c % TK); }

template <int PREC>
__device__ __forceinline__ void put_operand(void* va, void* vb, long idx, float v) {
  if constexpr (PREC == kBatchBF16x3) {
    const unsigned short h = bf16_bits(v);
    static_cast<unsigned short*>(va)[idx] = h;
    static_cast<unsigned short*>(vb)[idx] = bf16_bits(v - bf16_float(h));
  } else {
    static_cast<float*>(va)[idx] = v;
  }
}

// ------------------------------------------------------------------------------------------
// GEMM tile of TM instances x TNV matrix rows (TNV = 256, 128 or 64): four waves in a 2 x 2
// grid, each owning 64 instances x TNV/2 rows as 2 x BJ blocks of 32 x 32 accumulators (lane
// layout of v_mfma_f32_32x32x*). The larger tile reads fewer LDS bytes per product and fewer
// operand bytes per flop; which wins depends on how many tiles a problem has (the autotuner). Operand A rows are list positions (instances), B rows are matrix
// rows; both K-blocked (one K stage of a tile is one contiguous block).

template <int PREC, int TNV>
struct Smem;
template <int TNV>
struct Smem<kBatchBF16x3, TNV> {
  static constexpr int kRowsA = TM / 64, kRowsB = TNV / 64;  // rows tid/4 + 64 q, 8 bf16 each
  unsigned short a[2][2][TM][TK + PADB];                     // [stage][hi/lo][row][k]
  unsigned short b[2][2][TNV][TK + PADB];
};
template <int TNV>
struct Smem<kBatchF32, TNV> {
  static constexpr int kRowsA = TM / 32, kRowsB = TNV / 32;  // rows tid/8 + 32 q, 4 floats each
  float a[2][TM][TK + PADF];
  float b[2][TNV][TK + PADF];
};

template <int PREC>
__device__ __forceinline__ int loader_row(int q) {
  if constexpr (PREC == kBatchBF16x3)
    return threadIdx.x / 4 + 64 * q;
  else
    return threadIdx.x / 8 + 32 * q;
}

// One K stage of this thread's operand rows, held in registers between its global loads and
// its LDS stores (so that the loads of the next stages are in flight during the products).
template <int PREC, int TNV>
struct Frag;
template <int TNV>
struct Frag<kBatchBF16x3, TNV> {
  ushort8 a[2][TM / 64], b[2][TNV / 64];  // [hi/lo][row]
};
template <int TNV>
struct Frag<kBatchF32, TNV> {
  floatx4 a[TM / 32], b[TNV / 32];
};

// Loads never branch: a row outside the tile's valid range reads a valid dummy row (its
// products land in accumulator rows or columns that are discarded).
// aoff / boff: offsets of the thread's rows inside a K block; as / bs: elements per K block.
template <int PREC, int TNV>
__device__ __forceinline__ void fetch(Frag<PREC, TNV>& f, const void* Aa, const void* Ab, const void* Ba,
                                      const void* Bb, const long (&aoff)[Smem<PREC, TNV>::kRowsA],
                                      const long (&boff)[Smem<PREC, TNV>::kRowsB], long as, long bs, int stage) {
  constexpr int RA = Smem<PREC, TNV>::kRowsA, RB = Smem<PREC, TNV>::kRowsB;
  if constexpr (PREC == kBatchBF16x3) {
    const long ka = (long)stage * as + (threadIdx.x % 4) * 8, kb = (long)stage * bs + (threadIdx.x % 4) * 8;
#pragma unroll
    for (int h = 0; h < RA; ++h) {
      f.a[0][h] = *reinterpret_cast<const ushort8*>(static_cast<const unsigned short*>(Aa) + aoff[h] + ka);
      f.a[1][h] = *reinterpret_cast<const ushort8*>(static_cast<const unsigned short*>(Ab) + aoff[h] + ka);
    }
#pragma unroll
    for (int h = 0; h < RB; ++h) {
      f.b[0][h] = *reinterpret_cast<const ushort8*>(static_cast<const unsigned short*>(Ba) + boff[h] + kb);
      f.b[1][h] = *reinterpret_cast<const ushort8*>(static_cast<const unsigned short*>(Bb) + boff[h] + kb);
    }
  } else {
    const long ka = (long)stage * as + (threadIdx.x % 8) * 4, kb = (long)stage * bs + (threadIdx.x % 8) * 4;
#pragma unroll
    for (int h = 0; h < RA; ++h)
      f.a[h] = *reinterpret_cast<const floatx4*>(static_cast<const float*>(Aa) + aoff[h] + ka);
#pragma unroll
    for (int h = 0; h < RB; ++h)
      f.b[h] = *reinterpret_cast<const floatx4*>(static_cast<const float*>(Ba) + boff[h] + kb);
  }
}

// LDS stores of one stage; with MASK, matrix entries with k outside [kb, ke) become zero.
template <int PREC, int TNV, bool MASK>
__device__ __forceinline__ void stash(Smem<PREC, TNV>& sm, int buf, const Frag<PREC, TNV>& f, int stage, int kb,
                                      int ke) {
  constexpr int RA = Smem<PREC, TNV>::kRowsA, RB = Smem<PREC, TNV>::kRowsB;
  if constexpr (PREC == kBatchBF16x3) {
    const int kc = (threadIdx.x % 4) * 8;
    const int k0 = stage * TK + kc;
#pragma unroll
    for (int h = 0; h < RA; ++h)
#pragma unroll
      for (int p = 0; p < 2; ++p) *reinterpret_cast<ushort8*>(&sm.a[buf][p][loader_row<PREC>(h)][kc]) = f.a[p][h];
#pragma unroll
    for (int h = 0; h < RB; ++h)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        ushort8 bv = f.b[p][h];
        if constexpr (MASK) {
#pragma unroll
          for (int e = 0; e < 8; ++e) bv[e] = (k0 + e >= kb && k0 + e < ke) ? bv[e] : (unsigned short)0;
        }
        *reinterpret_cast<ushort8*>(&sm.b[buf][p][loader_row<PREC>(h)][kc]) = bv;
      }
  } else {
    const int kc = (threadIdx.x % 8) * 4;
    const int k0 = stage * TK + kc;
#pragma unroll
    for (int h = 0; h < RA; ++h) *reinterpret_cast<floatx4*>(&sm.a[buf][loader_row<PREC>(h)][kc]) = f.a[h];
#pragma unroll
    for (int h = 0; h < RB; ++h) {
      floatx4 bv = f.b[h];
      if constexpr (MASK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) bv[e] = (k0 + e >= kb && k0 + e < ke) ? bv[e] : 0.0f;
      }
      *reinterpret_cast<floatx4*>(&sm.b[buf][loader_row<PREC>(h)][kc]) = bv;
    }
  }
}

// Products of one LDS stage into this wave's 64 x TNV/2 part.
template <int PREC, int TNV>
__device__ __forceinline__ void compute(const Smem<PREC, TNV>& sm, int buf, floatx16 (&acc)[2][TNV / 64]) {
  constexpr int BJ = TNV / 64;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int wm = wave / 2, wn = wave % 2;
  if constexpr (PREC == kBatchBF16x3) {
#pragma unroll
    for (int kk = 0; kk < TK; kk += 16) {
      const int kq = kk + 8 * (lane / 32);
      bf16x8 fa[2][2], fb[BJ][2];  // [block][hi/lo]
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int p = 0; p < 2; ++p)
          fa[i][p] = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const ushort8*>(&sm.a[buf][p][wm * 64 + i * 32 + lane % 32][kq]));
#pragma unroll
      for (int j = 0; j < BJ; ++j)
#pragma unroll
        for (int p = 0; p < 2; ++p)
          fb[j][p] = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const ushort8*>(&sm.b[buf][p][wn * (TNV / 2) + j * 32 + lane % 32][kq]));
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][0], fb[j][0], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][1], fb[j][0], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][0], fb[j][1], acc[i][j], 0, 0, 0);
        }
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < TK; kk += 2) {
      const int kq = kk + lane / 32;
      float fa[2], fb[BJ];
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[i] = sm.a[buf][wm * 64 + i * 32 + lane % 32][kq];
#pragma unroll
      for (int j = 0; j < BJ; ++j) fb[j] = sm.b[buf][wn * (TNV / 2) + j * 32 + lane % 32][kq];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
  }
}

// acc = sum over k in [kb, ke) of A[row][k] B[col][k]. Stages of TK columns are double
// buffered in LDS and fetched into a ring of kRing (ring_of) register stages, so that the global
// loads run kRing - 1 stages ahead of the products. The stage count is rounded up to a multiple of
// kRing and every fetch is issued unconditionally (past the end it re-reads the last stage),
// so every step has the same instruction stream and the wait before an LDS store covers the
// loads of that stage only; a scheduling barrier keeps each fetch at the top of its step. The
// extra stages lie in the operands' zero padding (or are masked).
// The 256-row tile keeps a ring of two stages (its operand fragments take twice the registers).
template <int TNV>
constexpr int ring_of() {
  return TNV > 128 ? 2 : 4;
}
template <int PREC, int TNV, bool MASK>
__device__ __forceinline__ void tile_gemm(Smem<PREC, TNV>& sm, const void* Aa, const void* Ab, const void* Ba,
                                          const void* Bb, const long (&aoff)[Smem<PREC, TNV>::kRowsA],
                                          const long (&boff)[Smem<PREC, TNV>::kRowsB], long as, long bs, int kb,
                                          int ke, floatx16 (&acc)[2][TNV / 64]) {
  constexpr int kRing = ring_of<TNV>();
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < TNV / 64; ++j) acc[i][j] = floatx16{};
  const int s0 = kb / TK;
  int ns = (ke + TK - 1) / TK - s0;
  ns = (ns + kRing - 1) / kRing * kRing;
  // stage of visit position p (positions past the end re-read the last one)
  auto stage = [&](int p) { return s0 + min(p, ns - 1); };
  Frag<PREC, TNV> f[kRing];
#pragma unroll
  for (int r = 0; r < kRing; ++r) fetch<PREC, TNV>(f[r], Aa, Ab, Ba, Bb, aoff, boff, as, bs, stage(r));
  stash<PREC, TNV, MASK>(sm, 0, f[0], stage(0), kb, ke);
  __syncthreads();
  for (int p = 0; p < ns; p += kRing) {
#pragma unroll
    for (int r = 0; r < kRing; ++r) {
      // position p + r is in LDS buffer r & 1; f[r] is free again
      fetch<PREC, TNV>(f[r], Aa, Ab, Ba, Bb, aoff, boff, as, bs, stage(p + r + kRing));
      __builtin_amdgcn_sched_barrier(0);
      compute<PREC, TNV>(sm, r & 1, acc);
      stash<PREC, TNV, MASK>(sm, (r + 1) & 1, f[(r + 1) % kRing], stage(p + r + 1), kb, ke);
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------------------------------
// FP64 GEMM tile of the residual check and of the warm start's z = A x: T64 = 64 list positions
// x 64 matrix rows, K in stages of TK staged through LDS (double buffered, rows padded to
// TK + 2 doubles: the fragment reads of a half-wave hit distinct banks), four waves in a 2 x 2
// grid, each 32 x 32 as 2 x 2 blocks of v_mfma_f64_16x16x4f64 (lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16] of a 16 x 4 by 4 x 16 step, and D[l / 16 + 4 v][l % 16] in element v:
// checked on the device against a host product).
// Products of FP64 data with FP32 iterates are exact in FP64, so the sums are FP64 dot products.
constexpr int T64 = 64, PAD64 = 2;
typedef double doublex4 __attribute__((ext_vector_type(4)));
struct Smem64 {
  double a[2][T64][TK + PAD64];
  double b[2][T64][TK + PAD64];
};
// One K stage of this thread's chunks: 4 of the operand tile and 4 of the matrix tile, two
// doubles (16 bytes) each; chunk c = tid + 256 q covers row c / 16, columns 2 (c % 16) + {0, 1}.
struct Frag64 {
  double2 a[4], b[4];
};
__device__ __forceinline__ void fetch64(Frag64& f, const double* A, const double* Bm, long abase, long bbase, long as,
                                        long bs, int stage) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = threadIdx.x + BS * q, row = c >> 4, kc = (c & 15) * 2;
    f.a[q] = *reinterpret_cast<const double2*>(A + (long)stage * as + abase + (long)row * TK + kc);
    f.b[q] = *reinterpret_cast<const double2*>(Bm + (long)stage * bs + bbase + (long)row * TK + kc);
  }
}
// matrix entries with k outside [kb, ke) become zero
__device__ __forceinline__ void stash64(Smem64& sm, int buf, const Frag64& f, int stage, int kb, int ke) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = threadIdx.x + BS * q, row = c >> 4, kc = (c & 15) * 2, k0 = stage * TK + kc;
    double2 bv = f.b[q];
    bv.x = (k0 >= kb && k0 < ke) ? bv.x : 0.0;
    bv.y = (k0 + 1 >= kb && k0 + 1 < ke) ? bv.y : 0.0;
    *reinterpret_cast<double2*>(&sm.a[buf][row][kc]) = f.a[q];
    *reinterpret_cast<double2*>(&sm.b[buf][row][kc]) = bv;
  }
}
__device__ __forceinline__ void compute64(const Smem64& sm, int buf, doublex4 (&acc)[2][2]) {
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int wm = wave / 2, wn = wave % 2;
#pragma unroll
  for (int kk = 0; kk < TK; kk += 4) {
    double fa[2], fb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) fa[i] = sm.a[buf][wm * 32 + i * 16 + lane % 16][kk + lane / 16];
#pragma unroll
    for (int j = 0; j < 2; ++j) fb[j] = sm.b[buf][wn * 32 + j * 16 + lane % 16][kk + lane / 16];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
  }
}
// acc = sum over k in [kb, ke) of A[row][k] B[col][k] for the tile whose operand rows start at
// element abase and matrix rows at bbase of a K block (as / bs elements per K block). The next
// stage's loads are in flight while the current one is multiplied.
__device__ __forceinline__ void tile_gemm64(Smem64& sm, const double* A, const double* Bm, long abase, long bbase,
                                            long as, long bs, int kb, int ke, doublex4 (&acc)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int s0 = kb / TK, s1 = (ke + TK - 1) / TK;
  if (s1 <= s0) return;
  Frag64 f;
  fetch64(f, A, Bm, abase, bbase, as, bs, s0);
  stash64(sm, 0, f, s0, kb, ke);
  __syncthreads();
  for (int s = s0; s < s1; ++s) {
    const int buf = (s - s0) & 1;
    if (s + 1 < s1) fetch64(f, A, Bm, abase, bbase, as, bs, s + 1);
    compute64(sm, buf, acc);
    if (s + 1 < s1) stash64(sm, buf ^ 1, f, s + 1, kb, ke);
    __syncthreads();
  }
}
// Tile position of element v of FP64 block (i, j) for this lane: instance row, matrix column.
__device__ __forceinline__ int acc64_row(int wm, int i, int v, int lane) { return wm * 32 + i * 16 + lane / 16 + 4 * v; }
__device__ __forceinline__ int acc64_col(int wn, int j, int lane) { return wn * 32 + j * 16 + lane % 16; }

// Position in the tile of accumulator element v of block (i, j) for this lane.
__device__ __forceinline__ int acc_row(int wm, int i, int v, int lane) {
  return wm * 64 + i * 32 + 8 * (v / 4) + 4 * (lane / 32) + (v % 4);
}
template <int TNV>
__device__ __forceinline__ int acc_col(int wn, int j, int lane) {
  return wn * (TNV / 2) + j * 32 + lane % 32;
}

// M-tile descriptor: {penalty index, offset into lists, instance count}
struct MTile {
  int j, off, cnt;
};

template <int PREC, int TNV>
__device__ __forceinline__ void tile_offsets(const BatchArgs& a, const MTile& mt, int nt, long abase, long bbase,
                                             long (&aoff)[Smem<PREC, TNV>::kRowsA],
                                             long (&boff)[Smem<PREC, TNV>::kRowsB]) {
  // operand rows are list positions, matrix rows are rows; rows past the tile's instances or
  // past L hold other instances or zero padding (their results are discarded)
#pragma unroll
  for (int h = 0; h < Smem<PREC, TNV>::kRowsA; ++h) aoff[h] = abase + (long)(mt.off + loader_row<PREC>(h)) * TK;
#pragma unroll
  for (int h = 0; h < Smem<PREC, TNV>::kRowsB; ++h) boff[h] = bbase + (long)(nt * TNV + loader_row<PREC>(h)) * TK;
}

// XCD-aware walk over the grid of (M tile, N tile) pairs with N tiles in [n_begin, n_end).
// Workgroup g runs on XCD g % 8 (consecutive workgroups of a launch go round-robin over the
// eight XCDs); each XCD takes a contiguous range of M tiles (of N tiles when there are fewer M
// tiles than XCDs) and walks it with the M index fastest, so that the workgroups of one XCD
// work on a compact block of tiles at a time and share operand stages through its L2.
struct TileWalk {
  int per, count, mx, m0, n0, nmt;
  bool by_m;
  __device__ TileWalk(int nmt_, int n_begin, int n_end) : nmt(nmt_) {
    const int G = gridDim.x, x = blockIdx.x % 8, nn = n_end - n_begin;
    if (G % 8 != 0) {  // no XCD structure assumed: plain round robin
      per = G;
      by_m = true;
      m0 = 0;
      mx = nmt;
      n0 = n_begin;
      count = nmt * nn;
      return;
    }
    per = G / 8;
    by_m = nmt >= 8;
    if (by_m) {
      m0 = x * nmt / 8;
      mx = (x + 1) * nmt / 8 - m0;
      n0 = n_begin;
      count = mx * nn;
    } else {
      const int nb = n_begin + x * nn / 8, ne = n_begin + (x + 1) * nn / 8;
      m0 = 0;
      mx = nmt;
      n0 = nb;
      count = nmt * (ne - nb);
    }
  }
  // workgroup l of an XCD takes tiles l, l + per, ...
  __device__ int first() const { return gridDim.x % 8 != 0 ? blockIdx.x : blockIdx.x / 8; }
  __device__ int mt(int j) const { return m0 + j % mx; }
  __device__ int nt(int j) const { return n0 + j / mx; }
};

// Bucket sort of the slots in state `want` by penalty index into lists[] and the M-tile table
// (one workgroup). Before counting, slots in state `from` (if >= 0) move to state `to`. Slots
// are read in batches of kU per thread so that their loads overlap. The order inside a bucket
// is not fixed (atomic cursors); an instance's arithmetic does not depend on it.
constexpr int kU = 8;
__device__ void build_tiles(const BatchArgs& a, int* s_count /* LDS, kMaxRhoB */, int want, int from, int to) {
  const int tid = threadIdx.x, B = a.B;
  constexpr int kMaxRhoB = 64;
  __shared__ int s_cur[kMaxRhoB];
  if (tid < kMaxRhoB) s_count[tid] = 0;
  __syncthreads();
  for (int base = 0; base < B; base += BS * kU) {
    int st[kU], jj[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int b = min(base + u * BS + tid, B - 1);
      st[u] = a.status[b];
      jj[u] = a.jb[b];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int b = base + u * BS + tid;
      if (b >= B) continue;
      if (from >= 0 && st[u] == from) {
        a.status[b] = to;
        st[u] = to;
      }
      if (st[u] == want) atomicAdd(&s_count[jj[u]], 1);
    }
  }
  __syncthreads();
  if (tid == 0) {
    int off = 0, nt = 0;
    MTile* mt = reinterpret_cast<MTile*>(a.mtiles + 1);
    for (int j = 0; j < a.n_rho; ++j) {
      s_cur[j] = off;
      for (int c = 0; c < s_count[j]; c += TM) mt[nt++] = MTile{j, off + c, min(TM, s_count[j] - c)};
      off += s_count[j];
    }
    a.mtiles[0] = nt;
  }
  __syncthreads();
  for (int base = 0; base < B; base += BS * kU) {
    int st[kU], jj[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int b = min(base + u * BS + tid, B - 1);
      st[u] = a.status[b];
      jj[u] = a.jb[b];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int b = base + u * BS + tid;
      if (b < B && st[u] == want) {
        const int pos = atomicAdd(&s_cur[jj[u]], 1);
        a.lists[pos] = b;
        a.pos_of[b] = pos;
      }
    }
  }
  __syncthreads();
}

// Layer input w = [sigma x - q; rho z - y] of every running slot into operand parity `par`,
// kU elements per thread at a time (their loads overlap).
template <int PREC>
__device__ void layer_input(const BatchArgs& a, const float* s_rho, long vofs) {
  const int n = a.n, m = a.m, L = a.L;
  const long total = (long)a.B * L, gstride = (long)gridDim.x * BS;
  const float sigma = (float)a.sigma, eqs = (float)a.rho_eq_scale;
  for (long base = (long)blockIdx.x * BS + threadIdx.x; base < total; base += gstride * kU) {
    int st[kU], jj[kU], ps[kU];
    float u0[kU], u1[kU];
    unsigned char e[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long el = min(base + u * gstride, total - 1);
      const int b = (int)(el / L), r = (int)(el % L);
      const bool xr = r < n;
      const long xi = (long)b * n + (xr ? r : 0), zi = (long)b * m + (xr ? 0 : r - n);
      st[u] = a.status[b];
      jj[u] = a.jb[b];
      ps[u] = a.pos_of[b];
      e[u] = a.eq[xr ? 0 : r - n];
      u0[u] = xr ? a.X[xi] : a.Z[zi];
      u1[u] = xr ? a.Q[xi] : a.Y[zi];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long el = base + u * gstride;
      if (el >= total || st[u] != ST_RUNNING) continue;
      const int b = (int)(el / L), r = (int)(el % L);
      float w;
      if (r < n) {
        w = sigma * u0[u] - u1[u];
      } else {
        const float rho = s_rho[jj[u]] * (e[u] ? eqs : 1.0f);
        w = rho * u0[u] - u1[u];
      }
      put_operand<PREC>(a.Va, a.Vb, vofs + opidx(a.bpad, ps[u], r), w);
    }
  }
}

template <int PREC, int TNV>
__global__ void __launch_bounds__(BS) batch_kernel(BatchArgs a) {
  constexpr int BJ = TNV / 64;
  using SM = Smem<PREC, TNV>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  SM& sm = *reinterpret_cast<SM*>(smem_raw);
  Smem64& sm64 = *reinterpret_cast<Smem64*>(smem_raw);  // the FP64 phases (check, warm start)
  __shared__ int s_count[64];
  __shared__ int s_list[TM];   // instance ids of the current M tile
  __shared__ float s_rho[64];  // grid penalties in FP32
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wm = wave / 2, wn = wave % 2;
  const int G = gridDim.x, g = blockIdx.x;
  const int n = a.n, m = a.m, L = a.L, B = a.B;
  const long ldk = a.ldk;
  const long vpar = a.bpad * ldk;  // elements per parity of V
  const long as = a.bpad * TK, bs = a.lpad * TK;  // elements per K block of operands / matrices
  const int ntiles_n = (L + TNV - 1) / TNV;
  const float alpha = (float)a.alpha, oma = (float)(1.0 - a.alpha), sigma = (float)a.sigma;
  const float eqs = (float)a.rho_eq_scale;
  unsigned epoch = 0;
  const long gtid = (long)g * BS + tid, gstride = (long)G * BS;
  if (tid < a.n_rho) s_rho[tid] = (float)a.grid[tid];

  // M tile t's instance ids into s_list (entries past the tile's count repeat its first id)
  auto load_list = [&](const MTile& mt) {
    __syncthreads();  // the previous tile is done with s_list
    if (tid < TM) s_list[tid] = a.lists[mt.off + (tid < mt.cnt ? tid : 0)];
    __syncthreads();
  };

  // ---- admitted slots: cold ones start from zero, warm ones from their x and y with z = A x
  for (long b = gtid; b < B; b += gstride) {
    const int st = a.status[b];
    if (st == kSlotAdmitCold || st == kSlotAdmitWarm) a.iterations[b] = 0;
    if (st == kSlotAdmitCold) a.jb[b] = a.j0;
#pragma unroll
    for (int q = 0; q < 8; ++q) a.norms[b * 8 + q] = 0ull;
  }
  for (long base = gtid; base < (long)B * L; base += gstride * kU) {
    int st[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) st[u] = a.status[min(base + u * gstride, (long)B * L - 1) / L];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long el = base + u * gstride;
      if (el >= (long)B * L || st[u] != kSlotAdmitCold) continue;
      const int b = (int)(el / L), r = (int)(el % L);
      if (r < n) {
        a.X[(long)b * n + r] = 0.0f;
      } else {
        a.Z[(long)b * m + (r - n)] = 0.0f;
        a.Y[(long)b * m + (r - n)] = 0.0f;
      }
    }
  }
  if (!grid_barrier(a.bar, ++epoch)) return;
  if (g == 0) build_tiles(a, s_count, kSlotAdmitWarm, kSlotAdmitCold, ST_RUNNING);
  if (!grid_barrier(a.bar, ++epoch)) return;
  if (a.mtiles[0] > 0) {
    // warm start (Sec. II-B): check operand [x; y] of the warm slots at their list positions,
    // then z = A x from the z rows of the check product over K in [0, n)
    for (long base = gtid; base < (long)B * L; base += gstride * kU) {
      int st[kU], ps[kU];
      float xv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const long el = min(base + u * gstride, (long)B * L - 1);
        const int b = (int)(el / L), r = (int)(el % L);
        st[u] = a.status[b];
        ps[u] = a.pos_of[b];
        xv[u] = r < n ? a.X[(long)b * n + r] : a.Y[(long)b * m + (r - n)];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const long el = base + u * gstride;
        if (el >= (long)B * L || st[u] != kSlotAdmitWarm) continue;
        a.CVd[opidx(a.bpad, ps[u], (int)(el % L))] = (double)xv[u];
      }
    }
    if (!grid_barrier(a.bar, ++epoch)) return;
    const int nmt = a.mtiles[0];
    const MTile* mts = reinterpret_cast<const MTile*>(a.mtiles + 1);
    const TileWalk tw(2 * nmt, n / T64, (L + T64 - 1) / T64);  // 64-instance halves, constraint-row tiles
    for (int t = tw.first(); t < tw.count; t += tw.per) {
      const int u = tw.mt(t), half = u % 2;
      const MTile mt = mts[u / 2];
      const int cnt = mt.cnt - T64 * half;
      if (cnt <= 0) continue;  // the same for every thread of the workgroup
      const int r0 = tw.nt(t) * T64;
      load_list(mt);
      doublex4 acc[2][2];
      tile_gemm64(sm64, a.CVd, a.Cd, (long)(mt.off + T64 * half) * TK, (long)r0 * TK, as, bs, 0, n, acc);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int r = r0 + acc64_col(wn, j, lane);
          if (r < n || r >= L) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ti = acc64_row(wm, i, v, lane);
            if (ti < cnt) a.Z[(long)s_list[T64 * half + ti] * m + (r - n)] = (float)acc[i][j][v];
          }
        }
    }
    if (!grid_barrier(a.bar, ++epoch)) return;
  }
  if (g == 0) build_tiles(a, s_count, ST_RUNNING, kSlotAdmitWarm, ST_RUNNING);
  if (!grid_barrier(a.bar, ++epoch)) return;
  if (a.mtiles[0] == 0) return;  // nothing to run
  // ---- first layer input V_1 (parity 1)
  layer_input<PREC>(a, s_rho, vpar);
  if (!grid_barrier(a.bar, ++epoch)) return;

  const int ci = a.check_interval;
  for (int k = 1; k <= a.steps; ++k) {
    const bool is_check = (k % ci == 0) || (k == a.steps);
    const int nmt = a.mtiles[0];
    const MTile* mts = reinterpret_cast<const MTile*>(a.mtiles + 1);
    const long vin = (long)(k & 1) * vpar, vout = (long)((k + 1) & 1) * vpar;
    const TileWalk tw(nmt, 0, ntiles_n);

    // ---- layer GEMM + fused update
    for (int t = tw.first(); t < tw.count; t += tw.per) {
      const MTile mt = mts[tw.mt(t)];
      const int nt = tw.nt(t);
      load_list(mt);
      long aoff[SM::kRowsA], boff[SM::kRowsB];
      tile_offsets<PREC, TNV>(a, mt, nt, vin, (long)mt.j * a.w_stride, aoff, boff);
      floatx16 acc[2][BJ];
      tile_gemm<PREC, TNV, false>(sm, a.Va, a.Vb, a.Wa, a.Wb, aoff, boff, as, bs, 0, L, acc);
      const float rho_bar = s_rho[mt.j];
      // epilogue, one 32 x 32 block at a time: the 16 elements' state loads are issued
      // together, then the row-local update (relaxation, clamp, dual) and the stores
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
          const int r = nt * TNV + acc_col<TNV>(wn, j, lane);
          const bool rin = r < L, xr = r < n;
          const int ri = xr ? r : (rin ? r - n : 0);  // x index, or constraint index
          const float rho = rho_bar * (!xr && a.eq[ri] ? eqs : 1.0f);
          float u0[16], u1[16], u2[16], u3[16];
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const long b = s_list[acc_row(wm, i, v, lane)];
            const long xi = b * n + (xr ? ri : 0), zi = b * m + (xr ? 0 : ri);
            u0[v] = xr ? a.X[xi] : a.Z[zi];
            u1[v] = xr ? a.Q[xi] : a.Y[zi];
            u2[v] = a.Lo[zi];
            u3[v] = a.Up[zi];
          }
          if (!rin) continue;
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int ti = acc_row(wm, i, v, lane);
            if (ti >= mt.cnt) continue;
            const long b = s_list[ti];
            const float s = acc[i][j][v];
            float w, cv;
            if (xr) {
              const float x = alpha * s + oma * u0[v];
              a.X[b * n + ri] = x;
              w = sigma * x - u1[v];
              cv = x;
            } else {
              const float t2 = alpha * s + oma * u0[v] + u1[v] / rho;
              const float zn = t2 < u2[v] ? u2[v] : (t2 > u3[v] ? u3[v] : t2);
              const float yn = rho * (t2 - zn);
              a.Z[b * m + ri] = zn;
              a.Y[b * m + ri] = yn;
              w = rho * zn - yn;
              cv = yn;
            }
            const long oi = opidx(a.bpad, mt.off + ti, r);
            if (is_check)
              a.CVd[oi] = (double)cv;
            else
              put_operand<PREC>(a.Va, a.Vb, vout + oi, w);
          }
        }
    }
    if (!grid_barrier(a.bar, ++epoch)) return;
    if (!is_check) continue;

    // ---- check GEMM in FP64: [P, A'; A, 0] [x; y]; K split at n keeps P x and A'y apart, and
    // the constraint rows ([A, 0]) need only K in [0, n). The dual residual uses q rounded to
    // FP32 (the handle's copy): the published r_d adds that rounding (u |q_i|) and ||q|| drops it,
    // so the test passes only if the FP64 test with the caller's q does.
    {
      const double uq = 1.01 * 0x1p-24;
      const TileWalk tw64(2 * nmt, 0, (L + T64 - 1) / T64);
      for (int t = tw64.first(); t < tw64.count; t += tw64.per) {
        const int u = tw64.mt(t), half = u % 2;
        const MTile mt = mts[u / 2];
        const int cnt = mt.cnt - T64 * half;
        if (cnt <= 0) continue;  // the same for every thread of the workgroup
        const int r0 = tw64.nt(t) * T64;
        load_list(mt);
        const long abase = (long)(mt.off + T64 * half) * TK, bbase = (long)r0 * TK;
        doublex4 acc_p[2][2], acc_a[2][2];
        tile_gemm64(sm64, a.CVd, a.Cd, abase, bbase, as, bs, 0, n, acc_p);   // P x, A x
        tile_gemm64(sm64, a.CVd, a.Cd, abase, bbase, as, bs, n, r0 < n ? L : n, acc_a);  // A'y (x rows)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ti = acc64_row(wm, i, v, lane);
            const bool valid_i = ti < cnt;
            const long b = s_list[T64 * half + (valid_i ? ti : 0)];
            uint64_t nb[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              const int r = r0 + acc64_col(wn, j, lane);
              if (!valid_i || r >= L) continue;
              const double pp = acc_p[i][j][v];
              if (r < n) {
                const double pa = acc_a[i][j][v], q = (double)a.Q[b * n + r], dq = uq * fabs(q);
                const uint64_t vrd = abs_bits(fabs(pp + pa + q) + dq), vpx = abs_bits(pp), vat = abs_bits(pa);
                const uint64_t vq = abs_bits(lower_bound(fabs(q), dq));
                nb[N_RD] = vrd > nb[N_RD] ? vrd : nb[N_RD];
                nb[N_PX] = vpx > nb[N_PX] ? vpx : nb[N_PX];
                nb[N_ATY] = vat > nb[N_ATY] ? vat : nb[N_ATY];
                nb[N_Q] = vq > nb[N_Q] ? vq : nb[N_Q];
              } else {
                const double z = (double)a.Z[b * m + (r - n)];
                const uint64_t vrp = abs_bits(pp - z), vax = abs_bits(pp), vz = abs_bits(z);
                nb[N_RP] = vrp > nb[N_RP] ? vrp : nb[N_RP];
                nb[N_AX] = vax > nb[N_AX] ? vax : nb[N_AX];
                nb[N_Z] = vz > nb[N_Z] ? vz : nb[N_Z];
              }
            }
            // lanes with the same lane / 16 hold the same instance row: reduce over lane % 16
#pragma unroll
            for (int q = 0; q < 7; ++q) {
              uint64_t x = nb[q];
#pragma unroll
              for (int off = 1; off < 16; off <<= 1) {
                const uint64_t o = __shfl_xor(x, off, 64);
                x = o > x ? o : x;
              }
              nb[q] = x;
            }
            if (valid_i && (lane % 16) == 0) {
#pragma unroll
              for (int q = 0; q < 7; ++q)
                if (nb[q]) atomicMax(a.norms + b * 8 + q, (unsigned long long)nb[q]);
            }
          }
      }
    }
    if (!grid_barrier(a.bar, ++epoch)) return;

    // ---- per-instance decision (eqs. primal, dual, rho_update; nearest grid value)
    // host-mapped flag: one PCIe read per workgroup at every kAbortEvery-th check
    __shared__ int ab_s;
    if (tid == 0)
      ab_s = (k / ci) % kAbortEvery == kAbortEvery - 1 && a.abort_flag &&
             __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __syncthreads();
    const bool ab = ab_s != 0;
    for (long b = gtid; b < B; b += gstride) {
      if (a.status[b] != ST_RUNNING) continue;
      unsigned long long* nm = a.norms + b * 8;
      uint64_t bits[7];
      bool nonfinite = false;
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        bits[q] = nm[q];
        nm[q] = 0;
        nonfinite |= bits[q] >= kInfBits;
      }
      const double rp = bits_to_double(bits[N_RP]), rd = bits_to_double(bits[N_RD]);
      const double nax = bits_to_double(bits[N_AX]), nz = bits_to_double(bits[N_Z]);
      const double npx = bits_to_double(bits[N_PX]), naty = bits_to_double(bits[N_ATY]);
      const double nq = bits_to_double(bits[N_Q]);
      const int it = a.iterations[b] + k;  // iterations since admission
      int st = ST_RUNNING;
      if (nonfinite) {
        st = ST_NONFINITE;
      } else if (a.terminate) {
        const double eps_p = a.eps_abs + a.eps_rel * fmax(nax, nz);
        const double eps_d = a.eps_abs + a.eps_rel * fmax(fmax(npx, naty), nq);
        if (rp <= eps_p && rd <= eps_d) st = ST_SOLVED;
      }
      if (st == ST_RUNNING && it >= a.max_iter) st = ST_MAX_ITER;
      if (st == ST_RUNNING && ab) st = ST_ABORTED;
      int j = a.jb[b];
      if (st == ST_RUNNING && a.n_rho > 1 && rp > 0.0 && rd > 0.0) {
        const double num = rp * fmax(fmax(npx, naty), fmax(nq, 1e-4));
        const double den = rd * fmax(fmax(nax, nz), 1e-4);
        const double rh = a.grid[j] * sqrt(num / den);
        int jn = 0;
        while (jn < a.n_rho - 1 && rh > a.mid[jn]) ++jn;
        j = jn;
      }
      a.jb[b] = j;
      const int c = (it + ci - 1) / ci - 1;  // check number since admission
      if (c < a.max_checks) {
        if (a.rho_hist) a.rho_hist[b * a.max_checks + c] = j;
        if (a.prim_res) a.prim_res[b * a.max_checks + c] = rp;
        if (a.dual_res) a.dual_res[b * a.max_checks + c] = rd;
      }
      if (st != ST_RUNNING) {
        a.status[b] = st;
        a.iterations[b] = it;
      }
    }
    if (!grid_barrier(a.bar, ++epoch)) return;
    if (g == 0) build_tiles(a, s_count, ST_RUNNING, -1, -1);
    if (!grid_barrier(a.bar, ++epoch)) return;
    if (a.mtiles[0] == 0) return;
    if (k == a.steps) break;  // the next launch rebuilds the layer input from the state

    // ---- next layer input for the instances still running (penalty may have changed)
    layer_input<PREC>(a, s_rho, vout);
    if (!grid_barrier(a.bar, ++epoch)) return;
  }
  // slots still running carry their iteration count into the next launch
  for (long b = gtid; b < B; b += gstride)
    if (a.status[b] == ST_RUNNING) a.iterations[b] += a.steps;
}

}  // namespace

BatchPlan plan_batch(int prec, int tn) {
  BatchPlan p{nullptr, 0, 0, tn};
  const void* fn = nullptr;
  size_t smem = 0;
  if (prec == kBatchBF16x3 && tn == 128) {
    fn = reinterpret_cast<const void*>(&batch_kernel<kBatchBF16x3, 128>);
    smem = sizeof(Smem<kBatchBF16x3, 128>);
  } else if (prec == kBatchBF16x3 && tn == 64) {
    fn = reinterpret_cast<const void*>(&batch_kernel<kBatchBF16x3, 64>);
    smem = sizeof(Smem<kBatchBF16x3, 64>);
  } else if (prec == kBatchF32 && tn == 128) {
    fn = reinterpret_cast<const void*>(&batch_kernel<kBatchF32, 128>);
    smem = sizeof(Smem<kBatchF32, 128>);
  } else if (prec == kBatchF32 && tn == 64) {
    fn = reinterpret_cast<const void*>(&batch_kernel<kBatchF32, 64>);
    smem = sizeof(Smem<kBatchF32, 64>);
  } else if (prec == kBatchBF16x3 && tn == 256) {
    fn = reinterpret_cast<const void*>(&batch_kernel<kBatchBF16x3, 256>);
    smem = sizeof(Smem<kBatchBF16x3, 256>);
  } else if (prec == kBatchF32 && tn == 256) {
    fn = reinterpret_cast<const void*>(&batch_kernel<kBatchF32, 256>);
    smem = sizeof(Smem<kBatchF32, 256>);
  } else {
    return p;
  }
  smem = smem > sizeof(Smem64) ? smem : sizeof(Smem64);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess) return p;
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return p;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return p;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, BS, smem) != hipSuccess) return p;
  if (per_cu < 1) return p;
  p.fn = fn;
  p.grid = cus;  // one workgroup per compute unit
  p.smem = smem;
  return p;
}

hipError_t launch_batch(const BatchArgs& a, const BatchPlan& p, hipStream_t st) {
  if (!p.fn) return hipErrorInvalidValue;
  BatchArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(p.fn, dim3(p.grid), dim3(BS), args, p.smem, st);
}

namespace {
__global__ void fill_status_kernel(int B, int value, int* __restrict__ status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) status[b] = value;
}
__global__ void stage_kernel(int src, int n, int m, const float* __restrict__ X, const float* __restrict__ Y,
                             const int* __restrict__ jb, float* __restrict__ stage) {
  for (int i = threadIdx.x; i < n + m; i += blockDim.x)
    stage[i] = i < n ? X[(long)src * n + i] : Y[(long)src * m + (i - n)];
  if (threadIdx.x == 0) reinterpret_cast<int*>(stage)[n + m] = jb[src];
}
// one workgroup per listed slot
__global__ void admit_kernel(SlotList sl, int warm, int sx, int sy, int n, int m, float* __restrict__ X,
                             float* __restrict__ Y, int* __restrict__ jb, int* __restrict__ status,
                             const float* __restrict__ stage) {
  const long s = sl.s[blockIdx.x];
  if (warm) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) X[s * n + i] = i + sx < n ? stage[i + sx] : 0.0f;
    for (int i = threadIdx.x; i < m; i += blockDim.x) Y[s * m + i] = i + sy < m ? stage[n + i + sy] : 0.0f;
  }
  if (threadIdx.x == 0) {
    if (warm) jb[s] = reinterpret_cast<const int*>(stage)[n + m];
    status[s] = warm ? kSlotAdmitWarm : kSlotAdmitCold;
  }
}
// Parametric vectors of the listed slots (Sec. IV): q = F x0, l = lo - E x0, u = hi - E x0;
// one thread per (listed slot, row), one in-order FMA chain over the nx entries of x0 (the
// order of the tiled whole-batch update, so a slot gets the same vectors either way).
__global__ void __launch_bounds__(256) x0_slots_kernel(SlotList sl, int n, int m, int nx, const double* __restrict__ F,
                                                       const double* __restrict__ E, const double* __restrict__ lo,
                                                       const double* __restrict__ hi, const double* __restrict__ x0,
                                                       float* __restrict__ Q, float* __restrict__ Lo,
                                                       float* __restrict__ Up) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)sl.n * (n + m)) return;
  const int i = (int)(e / (n + m)), row = (int)(e % (n + m));
  const long s = sl.s[i];
  const double* arow = row < n ? F + (long)row * nx : E + (long)(row - n) * nx;
  const double* xi = x0 + (long)i * nx;
  double acc = 0.0;
  for (int c = 0; c < nx; ++c) acc = fma(arow[c], xi[c], acc);
  if (row < n) {
    Q[s * n + row] = (float)acc;
  } else {
    Lo[s * m + (row - n)] = (float)(lo[row - n] - acc);
    Up[s * m + (row - n)] = (float)(hi[row - n] - acc);
  }
}
// q, l, u rows of the listed slots from FP64 device arrays (n_slots x n, n_slots x m)
__global__ void vec_slots_kernel(SlotList sl, int n, int m, const double* __restrict__ q, const double* __restrict__ l,
                                 const double* __restrict__ u, float* __restrict__ Q, float* __restrict__ Lo,
                                 float* __restrict__ Up) {
  const int i = blockIdx.x;
  const long s = sl.s[i];
  for (int r = threadIdx.x; r < n + m; r += blockDim.x) {
    if (r < n) {
      if (q) Q[s * n + r] = (float)q[(long)i * n + r];
    } else {
      if (l) Lo[s * m + (r - n)] = (float)l[(long)i * m + (r - n)];
      if (u) Up[s * m + (r - n)] = (float)u[(long)i * m + (r - n)];
    }
  }
}
}  // namespace

hipError_t load_x0_slots(const SlotList& sl, int n, int m, int nx, const double* F, const double* E, const double* lo,
                         const double* hi, const double* x0, float* Q, float* Lo, float* Up, hipStream_t st) {
  if (sl.n <= 0) return hipSuccess;
  const long rows = (long)sl.n * (n + m);
  hipLaunchKernelGGL(x0_slots_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, sl, n, m, nx, F, E, lo,
                     hi, x0, Q, Lo, Up);
  return hipGetLastError();
}

hipError_t load_slots(const SlotList& sl, int n, int m, const double* q, const double* l, const double* u, float* Q,
                      float* Lo, float* Up, hipStream_t st) {
  if (sl.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(vec_slots_kernel, dim3((unsigned)sl.n), dim3(256), 0, st, sl, n, m, q, l, u, Q, Lo, Up);
  return hipGetLastError();
}

hipError_t fill_status(int B, int value, int* status, hipStream_t st) {
  hipLaunchKernelGGL(fill_status_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, B, value, status);
  return hipGetLastError();
}

hipError_t admit_slots(const SlotList& sl, int src, int sx, int sy, int n, int m, float* X, float* Y, int* jb,
                       int* status, float* stage, hipStream_t st) {
  if (sl.n <= 0) return hipSuccess;
  if (src >= 0) {
    hipLaunchKernelGGL(stage_kernel, dim3(1), dim3(256), 0, st, src, n, m, X, Y, jb, stage);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(admit_kernel, dim3((unsigned)sl.n), dim3(256), 0, st, sl, src != -1 ? 1 : 0, sx, sy, n, m, X, Y,
                     jb, status, stage);
  return hipGetLastError();
}

namespace {
// one thread per element of the blocked lpad x ldk destination
__global__ void split_kernel(long rows, int cols, const double* __restrict__ src, long ld_src,
                             unsigned short* __restrict__ hi, unsigned short* __restrict__ lo, long lpad, long ldk) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= lpad * ldk) return;
  const long blk = idx / (lpad * TK), rem = idx % (lpad * TK);
  const long r = rem / TK;
  const int c = (int)(blk * TK + rem % TK);
  if (r >= rows) {
    hi[idx] = 0;
    lo[idx] = 0;
    return;
  }
  const float v = c < cols ? (float)src[r * ld_src + c] : 0.0f;
  // split the FP64 value: hi from its FP32 rounding, lo from the remaining FP64 difference
  const unsigned short h = bf16_bits(v);
  const double diff = c < cols ? src[r * ld_src + c] - (double)bf16_float(h) : 0.0;
  hi[idx] = h;
  lo[idx] = bf16_bits((float)diff);
}
__global__ void pad64_kernel(long rows, int cols, const double* __restrict__ src, long ld_src,
                             double* __restrict__ dst, long lpad, long ldk) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= lpad * ldk) return;
  const long blk = idx / (lpad * TK), rem = idx % (lpad * TK);
  const long r = rem / TK;
  const int c = (int)(blk * TK + rem % TK);
  dst[idx] = (r < rows && c < cols) ? src[r * ld_src + c] : 0.0;
}
__global__ void pad_kernel(long rows, int cols, const double* __restrict__ src, long ld_src, float* __restrict__ dst,
                           long lpad, long ldk) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= lpad * ldk) return;
  const long blk = idx / (lpad * TK), rem = idx % (lpad * TK);
  const long r = rem / TK;
  const int c = (int)(blk * TK + rem % TK);
  dst[idx] = (r < rows && c < cols) ? (float)src[r * ld_src + c] : 0.0f;
}
}  // namespace


hipError_t split_bf16(long rows, int cols, const double* src, long ld_src, void* hi, void* lo, long lpad, long ldk,
                      hipStream_t st) {
  const long total = lpad * ldk;
  hipLaunchKernelGGL(split_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, rows, cols, src, ld_src,
                     static_cast<unsigned short*>(hi), static_cast<unsigned short*>(lo), lpad, ldk);
  return hipGetLastError();
}

hipError_t pad_f64(long rows, int cols, const double* src, long ld_src, double* dst, long lpad, long ldk,
                   hipStream_t st) {
  const long total = lpad * ldk;
  hipLaunchKernelGGL(pad64_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, rows, cols, src, ld_src,
                     dst, lpad, ldk);
  return hipGetLastError();
}

hipError_t pad_f32(long rows, int cols, const double* src, long ld_src, float* dst, long lpad, long ldk,
                   hipStream_t st) {
  const long total = lpad * ldk;
  hipLaunchKernelGGL(pad_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, rows, cols, src, ld_src,
                     dst, lpad, ldk);
  return hipGetLastError();
}

}  // namespace rqp
