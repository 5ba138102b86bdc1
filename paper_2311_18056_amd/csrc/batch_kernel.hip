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

#include <type_traits>

#include "device_common.h"

namespace rqp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));

// f(integral_constant<int, I>) for I in [I0, I1), unrolled at compile time.
template <int I0, int I1, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I0 < I1) {
    f(std::integral_constant<int, I0>{});
    static_for<I0 + 1, I1>(f);
  }
}

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
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned e) {
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
// The same with a 32-bit element index (idx * 4 < 2^32).
template <int PREC>
__device__ __forceinline__ void put_operand32(void* va, void* vb, unsigned idx, float v) {
  if constexpr (PREC == kBatchBF16x3) {
    const unsigned short h = bf16_bits(v);
    reinterpret_cast<unsigned short*>(static_cast<char*>(va) + idx * 2u)[0] = h;
    reinterpret_cast<unsigned short*>(static_cast<char*>(vb) + idx * 2u)[0] = bf16_bits(v - bf16_float(h));
  } else {
    reinterpret_cast<float*>(static_cast<char*>(va) + idx * 4u)[0] = v;
  }
}

// Element idx of an array addressed with a 32-bit byte offset (base in scalar registers, offset
// in one vector register): the caller guarantees idx * sizeof(T) < 2^32.
template <typename T>
__device__ __forceinline__ T& at32(T* base, unsigned idx) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T& at32(const T* base, unsigned idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(T));
}

// ------------------------------------------------------------------------------------------
// Operand staging. One K stage (TK = 32 columns) of a tile's operand rows goes from global
// memory straight into LDS through global_load_lds_dwordx4, without passing through registers:
// one wave instruction moves 64 chunks of 16 bytes to 1 KB of consecutive LDS bytes (lane i to
// bytes 16 i). A row of the stage (32 elements: 64, 128 or 256 bytes) stays whole, and its
// chunks are permuted by an XOR with a function of the row index (swz): lane i fetches the
// global chunk that belongs at LDS position i. The matrix-core fragment reads (one row per
// lane, the same chunk in all rows) then fall on distinct banks for every group of 8 or 16
// lanes. Loads never branch: rows past a tile's valid range read valid padding rows (their
// products land in results that are discarded).
typedef __attribute__((address_space(3))) void* lds_ptr_t;
template <int CPR>  // 16-byte chunks per row: 4 (BF16), 8 (FP32), 16 (FP64)
__device__ __forceinline__ int swz(int r) {
  if constexpr (CPR == 4)
    return ((r >> 1) ^ (r >> 2)) & 3;
  else if constexpr (CPR == 8)
    return (r ^ (r >> 3)) & 7;
  else
    return r & 15;
}
// ROWS rows of one K block starting at byte address src (rows CPR * 16 bytes apart) to lds.
template <int ROWS, int CPR>
__device__ __forceinline__ void dma_panel(const unsigned char* src, unsigned char* lds, int wave) {
  static_assert(ROWS * CPR % BS == 0, "a panel is a whole number of wave instructions per thread");
#pragma unroll
  for (int i = 0; i < ROWS * CPR / BS; ++i) {
    // instruction i covers rows [i BS / CPR, (i + 1) BS / CPR): a uniform base plus a lane offset
    const int ci = i * BS + threadIdx.x, row = ci / CPR, c = (ci % CPR) ^ swz<CPR>(row);
    const unsigned off = (unsigned)((row - i * (BS / CPR)) * (CPR * 16) + c * 16);
    __builtin_amdgcn_global_load_lds(src + i * BS * 16 + off, (lds_ptr_t)(lds + i * BS * 16 + wave * 1024), 16, 0, 0);
  }
}
template <int CPR>
__device__ __forceinline__ const unsigned char* frag_at(const unsigned char* panel, int row, int c) {
  return panel + row * (CPR * 16) + 16 * (c ^ swz<CPR>(row));
}
// Waits until at most N vector memory operations of this wave are outstanding (loads into LDS
// complete in issue order).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
// Workgroup barrier that the compiler does not move memory operations across.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}
// K loop over stages [s0, s1) with NST LDS buffers: the stages NST - 1 ahead are in flight while
// one is multiplied; one barrier per stage (stage s has landed for every wave, and every wave is
// done with the buffer that stage s + NST - 1 overwrites). issue(s, buf) starts the copy of
// stage s (LOADS instructions per thread); comp(s, buf) multiplies it. On entry the LDS buffers
// may still be read by the previous tile. Stores of the previous tile may still be in flight:
// the vector memory counter also counts them, but they were issued before every copy of this
// loop and copies complete in issue order, so "at most LOADS * k outstanding" still means that
// every copy but the last k stages' has landed. Loads of the caller must be complete on entry.
template <int NST, int LOADS, typename Issue, typename Comp>
__device__ __forceinline__ void kloop(int s0, int s1, unsigned char* lds, int stage_bytes, Issue&& issue, Comp&& comp) {
  static_assert(NST >= 2 && NST <= 4 && LOADS * (NST - 2) < 64, "pipeline depth");
  lds_barrier();
#pragma unroll
  for (int p = 0; p < NST - 1; ++p)
    if (s0 + p < s1) issue(s0 + p, lds + p * stage_bytes);
  for (int s = s0; s < s1; ++s) {
    const int ahead = min(s1 - 1 - s, NST - 2);  // stages issued after s
    if (NST >= 4 && ahead >= 2)
      wait_vm<LOADS*(NST >= 4 ? 2 : 0)>();
    else if (NST >= 3 && ahead >= 1)
      wait_vm<LOADS*(NST >= 3 ? 1 : 0)>();
    else
      wait_vm<0>();
    lds_barrier();
    const int q = s - s0;
    if (s + NST - 1 < s1) issue(s + NST - 1, lds + ((q + NST - 1) % NST) * stage_bytes);
    comp(s, lds + (q % NST) * stage_bytes);
  }
}

// ------------------------------------------------------------------------------------------
// Layer GEMM tile: TM instances (list positions) x TNV matrix rows (256, 128 or 64), four waves
// in a 2 x 2 grid, each owning 64 instances x TNV/2 rows as 2 x BJ blocks of 32 x 32
// accumulators (lane layout of v_mfma_f32_32x32x*). A stage holds the A rows (instances) then
// the B rows (matrix rows): BF16 high and low panels of 64-byte rows, or FP32 panels of 128-byte
// rows, (TM + TNV) x 128 bytes in both cases. A larger tile reads fewer LDS bytes per product
// and fewer operand bytes per flop; which wins depends on how many tiles a problem has (the
// autotuner).
template <int TNV>
struct LayerGeo {
  static constexpr int BJ = TNV / 64;
  static constexpr int STAGE = (TM + TNV) * 128;
  static constexpr int LOADS = STAGE / 16 / BS;
  static constexpr int NST = TNV >= 256 ? 3 : 4;
  static constexpr size_t SMEM = (size_t)NST * STAGE;
};

template <int PREC, int TNV>
__device__ __forceinline__ void layer_issue(const void* Aa, const void* Ab, const void* Ba, const void* Bb, long arow,
                                            long brow, long as, long bs, int s, unsigned char* buf, int wave) {
  if constexpr (PREC == kBatchBF16x3) {
    const long ao = ((long)s * as + arow * TK) * 2, bo = ((long)s * bs + brow * TK) * 2;
    dma_panel<TM, 4>(static_cast<const unsigned char*>(Aa) + ao, buf, wave);
    dma_panel<TM, 4>(static_cast<const unsigned char*>(Ab) + ao, buf + TM * 64, wave);
    dma_panel<TNV, 4>(static_cast<const unsigned char*>(Ba) + bo, buf + TM * 128, wave);
    dma_panel<TNV, 4>(static_cast<const unsigned char*>(Bb) + bo, buf + TM * 128 + TNV * 64, wave);
  } else {
    const long ao = ((long)s * as + arow * TK) * 4, bo = ((long)s * bs + brow * TK) * 4;
    dma_panel<TM, 8>(static_cast<const unsigned char*>(Aa) + ao, buf, wave);
    dma_panel<TNV, 8>(static_cast<const unsigned char*>(Ba) + bo, buf + TM * 128, wave);
  }
}

// Products of one stage into this wave's 64 x TNV/2 part. BF16: the three products
// hi*hi + lo*hi + hi*lo per k step of 16; lane l reads chunk 2 kk + l / 32 of its row (8
// elements), which is the k order of the 32x32x16 operand layout. FP32: lane l reads the chunk
// pair (2 g + l / 32) as four floats and feeds component s to the s-th of four 32x32x2
// products; A and B read the same chunks, so every product pairs equal k.
template <int PREC, int TNV>
__device__ __forceinline__ void layer_comp(const unsigned char* buf, floatx16 (&acc)[2][TNV / 64]) {
  constexpr int BJ = TNV / 64;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int wm = wave / 2, wn = wave % 2;
  if constexpr (PREC == kBatchBF16x3) {
    const unsigned char *ah = buf, *al = buf + TM * 64, *bh = buf + TM * 128, *bl = buf + TM * 128 + TNV * 64;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int c = 2 * kk + lane / 32;
      bf16x8 fa[2][2], fb[BJ][2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = wm * 64 + i * 32 + lane % 32;
        fa[i][0] = *reinterpret_cast<const bf16x8*>(frag_at<4>(ah, r, c));
        fa[i][1] = *reinterpret_cast<const bf16x8*>(frag_at<4>(al, r, c));
      }
#pragma unroll
      for (int j = 0; j < BJ; ++j) {
        const int r = wn * (TNV / 2) + j * 32 + lane % 32;
        fb[j][0] = *reinterpret_cast<const bf16x8*>(frag_at<4>(bh, r, c));
        fb[j][1] = *reinterpret_cast<const bf16x8*>(frag_at<4>(bl, r, c));
      }
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
    const unsigned char *pa = buf, *pb = buf + TM * 128;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int c = 2 * g + lane / 32;
      floatx4 fa[2], fb[BJ];
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[i] = *reinterpret_cast<const floatx4*>(frag_at<8>(pa, wm * 64 + i * 32 + lane % 32, c));
#pragma unroll
      for (int j = 0; j < BJ; ++j)
        fb[j] = *reinterpret_cast<const floatx4*>(frag_at<8>(pb, wn * (TNV / 2) + j * 32 + lane % 32, c));
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < BJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[i][s], fb[j][s], acc[i][j], 0, 0, 0);
    }
  }
}

// acc = sum over k in [0, L) of V[row][k] W[col][k] for the tile whose operand rows start at
// list position arow and matrix rows at brow; V and W are zero past column L.
template <int PREC, int TNV>
__device__ __forceinline__ void layer_tile(unsigned char* lds, const void* Aa, const void* Ab, const void* Ba,
                                           const void* Bb, long arow, long brow, long as, long bs, int L,
                                           floatx16 (&acc)[2][TNV / 64]) {
  using G = LayerGeo<TNV>;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < G::BJ; ++j) acc[i][j] = floatx16{};
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  kloop<G::NST, G::LOADS>(
      0, (L + TK - 1) / TK, lds, G::STAGE,
      [&](int s, unsigned char* buf) { layer_issue<PREC, TNV>(Aa, Ab, Ba, Bb, arow, brow, as, bs, s, buf, wave); },
      [&](int, const unsigned char* buf) { layer_comp<PREC, TNV>(buf, acc); });
}

// Position in the tile of accumulator element v of block (i, j) for this lane.
__device__ __forceinline__ int acc_row(int wm, int i, int v, int lane) {
  return wm * 64 + i * 32 + 8 * (v / 4) + 4 * (lane / 32) + (v % 4);
}
template <int TNV>
__device__ __forceinline__ int acc_col(int wn, int j, int lane) {
  return wn * (TNV / 2) + j * 32 + lane % 32;
}

// ------------------------------------------------------------------------------------------
// FP64 GEMM tile of the residual check and of the warm start's z = A x: T64 = 128 list
// positions x 128 matrix rows over one K range, four waves in a 2 x 2 grid, each 64 x 64 as
// 4 x 4 blocks of v_mfma_f64_16x16x4f64 (lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]
// of a 16 x 4 by 4 x 16 step, and D[l / 16 + 4 v][l % 16] in element v: checked on the device
// against a host product). A stage is the A rows then the B rows, 256-byte rows, two buffers.
// Lane group g = l / 16 reads chunk 4 h + g of its row (two doubles, k = 8 h + 2 g + {0, 1}) and
// feeds component s to the s-th of two products, so one read serves two products. Both operands
// are FP64 (the caller's data and exact copies of the returned FP32 values), so the sums are FP64
// dot products of what the solve returns.
constexpr int T64 = 128;
typedef double doublex4 __attribute__((ext_vector_type(4)));
struct CheckGeo {
  static constexpr int STAGE = 2 * T64 * 256;
  static constexpr int LOADS = STAGE / 16 / BS;
  static constexpr int NST = 2;
  static constexpr size_t SMEM = (size_t)NST * STAGE;
};
// acc = sum over the K stages [s0, s1) of A[row][k] B[col][k]; A rows start at list position arow,
// B rows at matrix row brow (as / bs: elements per K block). No masking: the A operands hold
// zeros wherever a tile's K range must not contribute (the x part and the y part of the check
// operand are separate, zero-padded arrays), so a non-finite iterate cannot leak in through a
// zero matrix entry and the stage loop is the same for every stage.
__device__ __forceinline__ void check_tile(unsigned char* lds, const double* A, const double* Bm, long arow, long brow,
                                           long as, long bs, int s0, int s1, doublex4 (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int lane = threadIdx.x % 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), wm = wave / 2, wn = wave % 2;
  kloop<CheckGeo::NST, CheckGeo::LOADS>(
      s0, s1, lds, CheckGeo::STAGE,
      [&](int s, unsigned char* buf) {
        dma_panel<T64, 16>(reinterpret_cast<const unsigned char*>(A + (long)s * as + arow * TK), buf, wave);
        dma_panel<T64, 16>(reinterpret_cast<const unsigned char*>(Bm + (long)s * bs + brow * TK), buf + T64 * 256,
                           wave);
      },
      [&](int, const unsigned char* buf) {
        const unsigned char *pa = buf, *pb = buf + T64 * 256;
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int c = 4 * h + lane / 16;
          double2 fa[4], fb[4];
#pragma unroll
          for (int i = 0; i < 4; ++i)
            fa[i] = *reinterpret_cast<const double2*>(frag_at<16>(pa, wm * 64 + i * 16 + lane % 16, c));
#pragma unroll
          for (int j = 0; j < 4; ++j)
            fb[j] = *reinterpret_cast<const double2*>(frag_at<16>(pb, wn * 64 + j * 16 + lane % 16, c));
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].x, fb[j].x, acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i].y, fb[j].y, acc[i][j], 0, 0, 0);
            }
        }
      });
}
// Tile position of element v of FP64 block (i, j) for this lane: instance row, matrix column.
__device__ __forceinline__ int acc64_row(int wm, int i, int v, int lane) { return wm * 64 + i * 16 + lane / 16 + 4 * v; }
__device__ __forceinline__ int acc64_col(int wn, int j, int lane) { return wn * 64 + j * 16 + lane % 16; }

// M-tile descriptor: {penalty index, offset into lists, instance count}
struct MTile {
  int j, off, cnt;
};

// XCD-aware walk over the grid of (M tile, N tile) pairs with N tiles in [n_begin, n_end).
// Workgroup g runs on XCD g % 8 (consecutive workgroups of a launch go round-robin over the
// eight XCDs); each XCD takes a contiguous range of M tiles (of N tiles when there are fewer M
// tiles than XCDs) and walks it with the M index fastest, so that the workgroups of one XCD
// work on a compact block of tiles at a time and share operand stages through its L2. When the
// M tiles do not split evenly over the XCDs, the XCD with the most of them can need more rounds
// of its workgroups than an even share of the pairs would (29 M tiles x 25 N tiles: 4 rounds
// where 3 suffice); then each XCD takes an equal contiguous range of the pairs in M-fastest
// order instead (balanced), which costs L2 locality, so only when it saves a round and only for
// the layer GEMM (may_balance): the FP64 check tiles read twice the operand bytes of a layer tile and
// measured no faster balanced.
struct TileWalk {
  int per, count, mx, m0, n0, p0;  // pair j of this XCD: M tile m0 + (p0 + j) % mx, N tile n0 + (p0 + j) / mx
  __device__ __forceinline__ TileWalk(int nmt, int n_begin, int n_end, bool may_balance = false) {
    const int G = gridDim.x, x = blockIdx.x % 8, nn = n_end - n_begin;
    p0 = 0;
    m0 = 0;
    mx = nmt;
    n0 = n_begin;
    if (G % 8 != 0) {  // no XCD structure assumed: plain round robin
      per = G;
      count = nmt * nn;
      return;
    }
    per = G / 8;
    bool bal = false;
    if (may_balance && nmt >= 8) {
      const int most = (nmt + 7) / 8 * nn, even = (nmt * nn + 7) / 8;  // pairs of the busiest XCD
      bal = (even + per - 1) / per < (most + per - 1) / per;
    }
    if (bal) {
      const int T = nmt * nn;
      p0 = x * T / 8;
      count = (x + 1) * T / 8 - p0;
    } else if (nmt >= 8) {
      m0 = x * nmt / 8;
      mx = (x + 1) * nmt / 8 - m0;
      count = mx * nn;
    } else {
      const int nb = n_begin + x * nn / 8, ne = n_begin + (x + 1) * nn / 8;
      n0 = nb;
      count = nmt * (ne - nb);
    }
  }
  // workgroup l of an XCD takes tiles l, l + per, ...
  __device__ int first() const { return gridDim.x % 8 != 0 ? blockIdx.x : blockIdx.x / 8; }
  __device__ int mt(int j) const { return m0 + (p0 + j) % mx; }
  __device__ int nt(int j) const { return n0 + (p0 + j) / mx; }
};

// Bucket sort of the slots in state `want` by penalty index into lists[] and the M-tile table
// (one workgroup). Before counting, slots in state `from` (if >= 0) move to state `to`. Slots
// are read in batches of kU per thread so that their loads overlap. The order inside a bucket
// is not fixed (atomic cursors); an instance's arithmetic does not depend on it.
constexpr int kU = 8;
template <typename AT>
__device__ __forceinline__ void build_tiles(const AT& a, int* s_count /* LDS, kMaxRhoB */, int want, int from, int to) {
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
template <int PREC, typename AT>
__device__ __forceinline__ void layer_input(const AT& a, const float* s_rho, long vofs) {
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

// The kernel reads its arguments through the kernarg segment pointer made opaque at the start of
// each phase (fresh), so the compiler loads the fields a phase needs where it needs them instead
// of keeping every field of the persistent loop in scalar registers (which spills).
typedef const __attribute__((address_space(4))) BatchArgs* cargs_t;
__device__ __forceinline__ cargs_t fresh(cargs_t p) {
  asm volatile("" : "+s"(p));
  return p;
}

template <int PREC, int TNV>
__global__ void __launch_bounds__(BS) batch_kernel(BatchArgs a_in) {
  (void)a_in;
  const cargs_t kp = (cargs_t)__builtin_amdgcn_kernarg_segment_ptr();
  const auto& a = *fresh(kp);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* const lds = smem_raw;  // operand stages of the layer and check GEMMs
  __shared__ int s_count[64];
  __shared__ int s_list[TM];   // instance ids of the current M tile
  __shared__ float s_rho[64];  // grid penalties in FP32
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wm = wave / 2, wn = wave % 2;
  const int G = gridDim.x, g = blockIdx.x;
  const int n = a.n, m = a.m, L = a.L, B = a.B;
  const long ldk = a.ldk;
  const long vpar = a.bpad * ldk;  // elements per parity of V
  const long cvy = a.bpad * ldk;   // the y part of the check operand follows the x part
  // elements per K block of the operands, the layer matrices and the check matrix
  const long as = a.bpad * TK, bs = a.lpad * TK, cs = a.cpad * TK;
  const int NX = (n + T64 - 1) / T64, NC = (m + T64 - 1) / T64;  // check row tiles: x rows, constraint rows
  // Row tiles of the layer GEMM: TNV rows each, except that the last TNV rows (or fewer) go in
  // tiles of TNS = TNV / 2 rows. The walks take row tiles in increasing order, so these come in
  // the last round of workgroups, which otherwise costs a whole round of TNV-row tiles however
  // few of them it holds (4096 instances x 3200 rows at 128 rows: 800 tiles, 32 in the fourth
  // round of 256 workgroups). Which rows a tile shape covers depends only on L and TNV, so an
  // instance's arithmetic is the same alone and in any batch.
  constexpr int TNS = TNV >= 128 ? TNV / 2 : TNV;
  static_assert(LayerGeo<TNS>::SMEM <= LayerGeo<TNV>::SMEM, "the small row tiles fit the large ones' LDS");
  const int nbig = TNV >= 128 ? (L - 1) / TNV : (L + TNV - 1) / TNV;
  const int ntiles_n = nbig + (L - nbig * TNV + TNS - 1) / TNS;
  const float alpha = (float)a.alpha, oma = (float)(1.0 - a.alpha), sigma = (float)a.sigma;
  const float eqs = (float)a.rho_eq_scale;
  unsigned epoch = 0;
  const long gtid = (long)g * BS + tid, gstride = (long)G * BS;
  if (tid < a.n_rho) s_rho[tid] = (float)a.grid[tid];

  // M tile t's instance ids into s_list (entries past the tile's count repeat its first id)
  auto load_list = [&](const int* lists, const MTile& mt) {
    __syncthreads();  // the previous tile is done with s_list
    if (tid < TM) s_list[tid] = lists[mt.off + (tid < mt.cnt ? tid : 0)];
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
  if (g == 0) build_tiles(*fresh(kp), s_count, kSlotAdmitWarm, kSlotAdmitCold, ST_RUNNING);
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
        const int r = (int)(el % L);
        if (r < n) a.CVd[opidx(a.bpad, ps[u], r)] = (double)xv[u] * (a.scl ? a.scl[2 * n + 2 * m + r] : 1.0);
      }
    }
    if (!grid_barrier(a.bar, ++epoch)) return;
    const int nmt = a.mtiles[0];
    const MTile* mts = reinterpret_cast<const MTile*>(a.mtiles + 1);
    const TileWalk tw(nmt, 0, NC);  // constraint-row tiles
    for (int t = tw.first(); t < tw.count; t += tw.per) {
      const auto& a = *fresh(kp);
      const MTile mt = mts[tw.mt(t)];
      const int r0 = n + tw.nt(t) * T64;
      load_list(a.lists, mt);
      doublex4 acc[4][4];
      check_tile(lds, a.CVd, a.Cd, mt.off, r0, as, cs, 0, (n + TK - 1) / TK, acc);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = r0 + acc64_col(wn, j, lane);
          if (r >= L) continue;
          const double fe = a.scl ? a.scl[r] : 1.0;  // E of constraint row r - n (zb = E A x)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ti = acc64_row(wm, i, v, lane);
            if (ti < mt.cnt) a.Z[(long)s_list[ti] * m + (r - n)] = (float)(acc[i][j][v] * fe);
          }
        }
    }
    if (!grid_barrier(a.bar, ++epoch)) return;
  }
  if (g == 0) build_tiles(*fresh(kp), s_count, ST_RUNNING, kSlotAdmitWarm, ST_RUNNING);
  if (!grid_barrier(a.bar, ++epoch)) return;
  if (a.mtiles[0] == 0) return;  // nothing to run
  // ---- first layer input V_1 (parity 1)
  layer_input<PREC>(*fresh(kp), s_rho, vpar);
  if (!grid_barrier(a.bar, ++epoch)) return;

  const int ci = a.check_interval;
  for (int k = 1; k <= a.steps; ++k) {
    const auto& a = *fresh(kp);
    const bool is_check = (k % ci == 0) || (k == a.steps);
    const int nmt = a.mtiles[0];
    const MTile* mts = reinterpret_cast<const MTile*>(a.mtiles + 1);
    const long vin = (long)(k & 1) * vpar, vout = (long)((k + 1) & 1) * vpar;
    const TileWalk tw(nmt, 0, ntiles_n, true);

    // ---- layer GEMM + fused update: one tile of TR rows starting at matrix row r0
    auto layer_step = [&](auto TRc, int mti, int r0) __attribute__((always_inline)) {
      constexpr int TR = decltype(TRc)::value, BJR = TR / 64;
      const auto& a = *fresh(kp);
      const MTile mt = mts[mti];
      load_list(a.lists, mt);
      constexpr long es = PREC == kBatchBF16x3 ? 2 : 4;
      const unsigned char* Aa = static_cast<const unsigned char*>(a.Va) + vin * es;
      const unsigned char* Ab = a.Vb ? static_cast<const unsigned char*>(a.Vb) + vin * es : nullptr;
      const unsigned char* Ba = static_cast<const unsigned char*>(a.Wa) + (long)mt.j * a.w_stride * es;
      const unsigned char* Bb = a.Wb ? static_cast<const unsigned char*>(a.Wb) + (long)mt.j * a.w_stride * es : nullptr;
      floatx16 acc[2][BJR];
      layer_tile<PREC, TR>(lds, Aa, Ab, Ba, Bb, mt.off, (long)r0, as, bs, L, acc);
      const float rho_bar = s_rho[mt.j];
      // epilogue, one 32 x 32 block at a time (block indices are compile-time constants, so the
      // accumulators stay in registers). A lane's 16 elements of a block share its column r (one
      // layer row) and take 16 instances; the instances' state offsets are formed once per
      // block row i. All state loads of a block are issued together, then the row-local update
      // (relaxation, clamp, dual) and the stores; elements past the tile's instance count load
      // valid rows (the list repeats its first id) and store nothing. Offsets are 32-bit
      // (B * max(n, m) and the operand size, in bytes, are checked at setup).
      const auto& ae = *fresh(kp);
      unsigned char* const vo = static_cast<unsigned char*>(ae.Va) + vout * (PREC == kBatchBF16x3 ? 2 : 4);
      unsigned char* const vo2 = ae.Vb ? static_cast<unsigned char*>(ae.Vb) + vout * 2 : nullptr;
      static_for<0, 2>([&](auto I) {
        constexpr int i = decltype(I)::value;
        unsigned on[16], om[16], oo[16];
        bool ok[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int ti = acc_row(wm, i, v, lane);
          const unsigned b = (unsigned)s_list[ti];
          on[v] = b * (unsigned)n;
          om[v] = b * (unsigned)m;
          oo[v] = (unsigned)ti * TK;
          ok[v] = ti < mt.cnt;
        }
        static_for<0, BJR>([&](auto J) {
          constexpr int j = decltype(J)::value;
          const int r = r0 + acc_col<TR>(wn, j, lane);
          if (r >= L) return;
          // operand index of element v: obase + oo[v] (K-blocked, list position mt.off + ti)
          const unsigned obase = ((unsigned)(r / TK) * (unsigned)ae.bpad + (unsigned)mt.off) * TK + (unsigned)(r % TK);
          if (r < n) {
            // check operand: x in original units, rounded as the output is
            const double fx = ae.scl ? ae.scl[2 * n + 2 * m + r] : 1.0;
            float xo[16], qv[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              xo[v] = at32(ae.X, on[v] + r);
              qv[v] = at32(ae.Q, on[v] + r);
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const float x = alpha * acc[i][j][v] + oma * xo[v];
              if (!ok[v]) continue;
              at32(ae.X, on[v] + r) = x;
              if (is_check)
                at32(ae.CVd, obase + oo[v]) = (double)(float)((double)x * fx);
              else
                put_operand32<PREC>(vo, vo2, obase + oo[v], sigma * x - qv[v]);
            }
          } else {
            const int ri = r - n;
            const float rho = rho_bar * (ae.eq[ri] ? eqs : 1.0f), rinv = 1.0f / rho;
            const double fy = ae.scl ? ae.scl[3 * n + 2 * m + ri] : 1.0;
            float zo[16], yo[16], lo[16], up[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              zo[v] = at32(ae.Z, om[v] + ri);
              yo[v] = at32(ae.Y, om[v] + ri);
              lo[v] = at32(ae.Lo, om[v] + ri);
              up[v] = at32(ae.Up, om[v] + ri);
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const float t2 = alpha * acc[i][j][v] + oma * zo[v] + yo[v] * rinv;
              const float zn = t2 < lo[v] ? lo[v] : (t2 > up[v] ? up[v] : t2);
              const float yn = rho * (t2 - zn);
              if (!ok[v]) continue;
              at32(ae.Z, om[v] + ri) = zn;
              at32(ae.Y, om[v] + ri) = yn;
              if (is_check)
                at32(ae.CVd + cvy, obase + oo[v]) = (double)(float)((double)yn * fy);
              else
                put_operand32<PREC>(vo, vo2, obase + oo[v], rho * zn - yn);
            }
          }
        });
      });
    };
    for (int t = tw.first(); t < tw.count; t += tw.per) {
      const int nt = tw.nt(t);
      if (nt < nbig)
        layer_step(std::integral_constant<int, TNV>{}, tw.mt(t), nt * TNV);
      else
        layer_step(std::integral_constant<int, TNS>{}, tw.mt(t), nbig * TNV + (nt - nbig) * TNS);
    }
    if (!grid_barrier(a.bar, ++epoch)) return;
    if (!is_check) continue;

    // ---- check GEMM in FP64: [P, A'; A, 0] [x; y] as three kinds of tiles, each over one K
    // range with one accumulator: P x (x rows, K in [0, n)), A'y (x rows, K in [n, L)) and A x
    // (constraint rows, K in [0, n)). P x and A'y go to per-position buffers (the dual residual
    // needs their sum, the tolerance each norm); the A x tiles finish the primal side at once.
    {
      const TileWalk tw64(nmt, 0, 2 * NX + NC);
      for (int t = tw64.first(); t < tw64.count; t += tw64.per) {
        const auto& a = *fresh(kp);
        const MTile mt = mts[tw64.mt(t)];
        const int u = tw64.nt(t);
        const int kind = u < NX ? 0 : (u < 2 * NX ? 1 : 2);  // P x, A'y, A x (one kind per workgroup)
        const int r0 = kind == 2 ? n + (u - 2 * NX) * T64 : (u - kind * NX) * T64;
        load_list(a.lists, mt);
        doublex4 acc[4][4];
        check_tile(lds, kind == 1 ? a.CVd + cvy : a.CVd, a.Cd, mt.off, r0, as, cs, kind == 1 ? n / TK : 0,
                   kind == 1 ? (L + TK - 1) / TK : (n + TK - 1) / TK, acc);
        double* const R = kind == 0 ? a.Rpx : a.Raty;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ti = acc64_row(wm, i, v, lane);
            const bool valid_i = ti < mt.cnt;
            const long b = s_list[valid_i ? ti : 0];
            uint64_t nb[3] = {0, 0, 0};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int r = r0 + acc64_col(wn, j, lane);
              const double pv = acc[i][j][v];
              if (kind < 2) {
                if (!valid_i || r >= n) continue;
                R[(long)(mt.off + ti) * n + r] = pv;
                const uint64_t vb = abs_bits(pv);
                nb[0] = vb > nb[0] ? vb : nb[0];
              } else {
                if (!valid_i || r >= L) continue;
                // z in original units, rounded as the output is
                const double z = (double)(float)((double)a.Z[b * m + (r - n)] * (a.scl ? a.scl[n + m + r] : 1.0));
                const uint64_t vrp = abs_bits(pv - z), vax = abs_bits(pv), vz = abs_bits(z);
                nb[0] = vrp > nb[0] ? vrp : nb[0];
                nb[1] = vax > nb[1] ? vax : nb[1];
                nb[2] = vz > nb[2] ? vz : nb[2];
              }
            }
            // lanes with the same lane / 16 hold the same instance row: reduce over lane % 16
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              uint64_t x = nb[q];
#pragma unroll
              for (int off = 1; off < 16; off <<= 1) {
                const uint64_t o = __shfl_xor(x, off, 64);
                x = o > x ? o : x;
              }
              nb[q] = x;
            }
            if (valid_i && (lane % 16) == 0) {
              unsigned long long* nm = a.norms + b * 8;
              if (kind == 0) {
                if (nb[0]) atomicMax(nm + N_PX, (unsigned long long)nb[0]);
              } else if (kind == 1) {
                if (nb[0]) atomicMax(nm + N_ATY, (unsigned long long)nb[0]);
              } else {
                if (nb[0]) atomicMax(nm + N_RP, (unsigned long long)nb[0]);
                if (nb[1]) atomicMax(nm + N_AX, (unsigned long long)nb[1]);
                if (nb[2]) atomicMax(nm + N_Z, (unsigned long long)nb[2]);
              }
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
    // one wave per instance: the dual residual and ||q|| from the P x and A'y rows of the
    // instance's list position and its q (the handle's FP32 copy: the published r_d adds that
    // rounding, u |q_i|, and ||q|| drops it, so the test passes only if the FP64 test with the
    // caller's q does), then lane 0 decides
    const double uq = 1.01 * 0x1p-24;
    const long gw = (long)g * (BS / 64) + wave, nw = (long)G * (BS / 64);
    for (long b = gw; b < B; b += nw) {
      const auto& a = *fresh(kp);
      if (a.status[b] != ST_RUNNING) continue;  // the same for every lane of the wave
      const long pos = a.pos_of[b];
      const double* const px = a.Rpx + pos * n;
      const double* const pa = a.Raty + pos * n;
      const float* const qb = a.Q + b * n;
      const double* const sq = a.scl ? a.scl + n + m : nullptr;  // 1 / (c D): q = qb / (c D)
      uint64_t vrd = 0, vq = 0;
      // kDecRows rows per lane and pass, all loads of a pass issued before any use
      constexpr int kDecRows = 8;
      for (int r0 = 0; r0 < n; r0 += 64 * kDecRows) {
        double pv[kDecRows], av[kDecRows], qv[kDecRows];
#pragma unroll
        for (int u = 0; u < kDecRows; ++u) {
          const int r = r0 + lane + 64 * u;
          const bool in = r < n;
          pv[u] = in ? px[r] : 0.0;
          av[u] = in ? pa[r] : 0.0;
          qv[u] = in ? (double)qb[r] * (sq ? sq[r] : 1.0) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kDecRows; ++u) {
          const double dq = uq * fabs(qv[u]);
          const uint64_t x1 = abs_bits(fabs(pv[u] + av[u] + qv[u]) + dq), x2 = abs_bits(lower_bound(fabs(qv[u]), dq));
          vrd = x1 > vrd ? x1 : vrd;
          vq = x2 > vq ? x2 : vq;
        }
      }
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint64_t o1 = __shfl_xor(vrd, off, 64), o2 = __shfl_xor(vq, off, 64);
        vrd = o1 > vrd ? o1 : vrd;
        vq = o2 > vq ? o2 : vq;
      }
      if (lane != 0) continue;
      unsigned long long* nm = a.norms + b * 8;
      uint64_t bits[7];
      bool nonfinite = false;
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        bits[q] = q == N_RD ? vrd : (q == N_Q ? vq : (uint64_t)nm[q]);
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
    if (g == 0) build_tiles(*fresh(kp), s_count, ST_RUNNING, -1, -1);
    if (!grid_barrier(a.bar, ++epoch)) return;
    if (a.mtiles[0] == 0) return;
    if (k == a.steps) break;  // the next launch rebuilds the layer input from the state

    // ---- next layer input for the instances still running (penalty may have changed)
    layer_input<PREC>(*fresh(kp), s_rho, vout);
    if (!grid_barrier(a.bar, ++epoch)) return;
  }
  // slots still running carry their iteration count into the next launch
  for (long b = gtid; b < B; b += gstride)
    if (a.status[b] == ST_RUNNING) a.iterations[b] += a.steps;
}

template <int TNV>
constexpr size_t kernel_smem() {
  return LayerGeo<TNV>::SMEM > CheckGeo::SMEM ? LayerGeo<TNV>::SMEM : CheckGeo::SMEM;
}

}  // namespace

size_t batch_smem(int prec, int tn) {
  (void)prec;
  return tn == 256 ? kernel_smem<256>() : tn == 128 ? kernel_smem<128>() : tn == 64 ? kernel_smem<64>() : 0;
}

namespace {
const void* batch_fn(int prec, int tn) {
  if (prec == kBatchBF16x3) {
    if (tn == 256) return reinterpret_cast<const void*>(&batch_kernel<kBatchBF16x3, 256>);
    if (tn == 128) return reinterpret_cast<const void*>(&batch_kernel<kBatchBF16x3, 128>);
    if (tn == 64) return reinterpret_cast<const void*>(&batch_kernel<kBatchBF16x3, 64>);
  } else if (prec == kBatchF32) {
    if (tn == 256) return reinterpret_cast<const void*>(&batch_kernel<kBatchF32, 256>);
    if (tn == 128) return reinterpret_cast<const void*>(&batch_kernel<kBatchF32, 128>);
    if (tn == 64) return reinterpret_cast<const void*>(&batch_kernel<kBatchF32, 64>);
  }
  return nullptr;
}
}  // namespace

BatchPlan plan_batch(int prec, int tn) {
  BatchPlan p{nullptr, 0, 0, tn};
  const void* fn = batch_fn(prec, tn);
  const size_t smem = batch_smem(prec, tn);
  if (!fn || !smem) return p;
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
                             const float* __restrict__ stage, const double* __restrict__ scl) {
  const long s = sl.s[blockIdx.x];
  if (warm) {
    // scaled state: a shifted entry changes rows, so it changes units (D for x, E / c for y)
    const double* fx = scl && sx ? scl + 2 * n + 2 * m : nullptr;
    const double* fy = scl && sy ? scl + 3 * n + 2 * m : nullptr;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      X[s * n + i] = i + sx >= n ? 0.0f : fx ? (float)((double)stage[i + sx] * fx[i + sx] / fx[i]) : stage[i + sx];
    for (int i = threadIdx.x; i < m; i += blockDim.x)
      Y[s * m + i] = i + sy >= m ? 0.0f
                     : fy ? (float)((double)stage[n + i + sy] * fy[i + sy] / fy[i])
                          : stage[n + i + sy];
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
// (scaled with Ruiz scaling: c D q, E l, E u)
__global__ void vec_slots_kernel(SlotList sl, int n, int m, const double* __restrict__ q, const double* __restrict__ l,
                                 const double* __restrict__ u, float* __restrict__ Q, float* __restrict__ Lo,
                                 float* __restrict__ Up, const double* __restrict__ scl) {
  const int i = blockIdx.x;
  const long s = sl.s[i];
  for (int r = threadIdx.x; r < n + m; r += blockDim.x) {
    const double f = scl ? scl[r] : 1.0;  // c D_r, or E of constraint row r - n
    if (r < n) {
      if (q) Q[s * n + r] = (float)(f * q[(long)i * n + r]);
    } else {
      if (l) Lo[s * m + (r - n)] = (float)(f * l[(long)i * m + (r - n)]);
      if (u) Up[s * m + (r - n)] = (float)(f * u[(long)i * m + (r - n)]);
    }
  }
}
// One thread per output element: x = D xb, z = zb (1 / E), y = yb (E / c), each FP32 from the
// FP64 product (the same operations the check applies to its operands).
__global__ void unscale_kernel(long B, int n, int m, const float* __restrict__ X, const float* __restrict__ Z,
                               const float* __restrict__ Y, const double* __restrict__ scl, float* __restrict__ x,
                               float* __restrict__ z, float* __restrict__ y) {
  const long per = (long)n + 2L * m, e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * per) return;
  const long b = e / per;
  const int r = (int)(e % per);
  if (r < n) {
    x[b * n + r] = (float)((double)X[b * n + r] * scl[2 * n + 2 * m + r]);
  } else if (r < n + m) {
    const int i = r - n;
    z[b * m + i] = (float)((double)Z[b * m + i] * scl[2 * n + m + i]);
  } else {
    const int i = r - n - m;
    y[b * m + i] = (float)((double)Y[b * m + i] * scl[3 * n + 2 * m + i]);
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
                      float* Lo, float* Up, const double* scl, hipStream_t st) {
  if (sl.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(vec_slots_kernel, dim3((unsigned)sl.n), dim3(256), 0, st, sl, n, m, q, l, u, Q, Lo, Up, scl);
  return hipGetLastError();
}

hipError_t unscale_outputs(int B, int n, int m, const float* X, const float* Z, const float* Y, const double* scl,
                           float* x, float* z, float* y, hipStream_t st) {
  const long total = (long)B * ((long)n + 2L * m);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(unscale_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, (long)B, n, m, X, Z, Y,
                     scl, x, z, y);
  return hipGetLastError();
}

hipError_t fill_status(int B, int value, int* status, hipStream_t st) {
  hipLaunchKernelGGL(fill_status_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, B, value, status);
  return hipGetLastError();
}

hipError_t admit_slots(const SlotList& sl, int src, int sx, int sy, int n, int m, float* X, float* Y, int* jb,
                       int* status, float* stage, const double* scl, hipStream_t st) {
  if (sl.n <= 0) return hipSuccess;
  if (src >= 0) {
    hipLaunchKernelGGL(stage_kernel, dim3(1), dim3(256), 0, st, src, n, m, X, Y, jb, stage);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(admit_kernel, dim3((unsigned)sl.n), dim3(256), 0, st, sl, src != -1 ? 1 : 0, sx, sy, n, m, X, Y,
                     jb, status, stage, scl);
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
