// Persistent ReLU-QP layer kernel for gfx950: every iteration, check and penalty switch of
// Algorithm 1 (online stage) in one cooperative launch.
//
// Iteration (Sec. III-A; OSQP over-relaxation alpha; alpha = 1 is the paper's layer). With
// w = [sigma x - q ; rho z - y] and the compact layer matrix
//     Wc_j = [I; A] D_j [I, A'] = [D_j, D_j A'; A D_j, A D_j A'],   D_j = (P + sigma I + A' rho_j A)^-1,
// one matvec gives both xt = D_j (sigma x - q + A'(rho z - y)) and s = A xt. Then
//     x <- alpha xt + (1 - alpha) x
//     t  = alpha s + (1 - alpha) z + y / rho,   z <- clamp(t, l, u),   y <- rho (t - z)
// are row-local, and the next w is row-local too. This is the paper's "v <- clamp(W v + b)"
// (eq. gpu_update) with an (n+m)^2 weight instead of its (n+2m)^2 one: the paper's W also
// precomputes the products of D with A.
//
// Parallel layout: workgroup g owns a contiguous block of rows of Wc (row-parallel, Sec.
// III-A). Lane t of a workgroup owns the columns c = t + 1024 k of every row of the block and
// keeps the first NRS rows of its columns in registers for the whole solve (reloaded only
// when the penalty changes); further rows stream from memory. After the row-local update each
// row owner publishes its entry of the next w as an 8-byte {value, tag} word; every lane polls
// the words of its own columns until the tags match. That single round trip is both the data
// exchange and the synchronisation: there is no grid barrier.
//
// Every check_interval iterations (Sec. III-C) the owners publish [x; y], every workgroup
// forms its rows of [P, A'; A, 0][x; y] with FP64 accumulation, reduces seven inf-norms as
// ordered bit patterns (exact and order-independent, NaN-propagating), publishes them, and
// every workgroup reduces all partials itself. All workgroups therefore take bit-identical
// decisions (eqs. primal, dual and rho_update) without a broadcast.
#include "layer_kernel.h"

#include "device_common.h"

namespace rqp {
namespace {

constexpr int BS = kLayerBlock;
constexpr int NWAVE = BS / kWave;
constexpr unsigned kSpinLimit = 1u << 22;

enum { ST_RUNNING = 0, ST_SOLVED = 1, ST_MAX_ITER = 2, ST_NONFINITE = 3, ST_ABORTED = 4, ST_INTERNAL = 5 };
constexpr int kMaxRho = 64;  // the host accepts at most 64 penalty values

// penalty grid and the geometric midpoints between neighbours, copied to LDS once per launch
struct RhoTable {
  double grid[kMaxRho];
  double mid[kMaxRho];
};
enum { N_RP = 0, N_RD, N_AX, N_Z, N_PX, N_ATY, N_Q, N_FLAGS };

// The error word holds the tag of the solve that failed, so a failure never leaks into a later
// solve (each solve has its own tag range).
__device__ __forceinline__ bool err_set(const unsigned* err, uint32_t tag) {
  return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == tag;
}
__device__ __forceinline__ void err_raise(unsigned* err, uint32_t tag) {
  __hip_atomic_store(err, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Poll the exchange words of this lane's columns until every tag equals `tag`.
template <typename T, int NC>
__device__ __forceinline__ bool gather(const uint64_t* buf, int L, uint32_t tag, T (&v)[NC], const unsigned* err,
                                       uint32_t etag) {
  constexpr int NW = LLWords<T>::kWords;
  uint64_t w[NC][NW];
  const int tid = threadIdx.x;
  const uint64_t dummy = (uint64_t)tag << 32;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int c = tid + BS * k;
#pragma unroll
    for (int q = 0; q < NW; ++q) w[k][q] = (c < L) ? ll_load_word(buf + (long)c * NW + q) : dummy;
  }
  unsigned spins = 0;
  bool ok = true;
  while (true) {
    bool all = true;
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int q = 0; q < NW; ++q) all &= ll_tag(w[k][q]) == tag;
    if (all) break;
    // a short pause between polls (about 0.1 us) thins the polling traffic of all workgroups on
    // the fabric while the producers' stores travel (1 % faster per iteration than polling back
    // to back; longer pauses lose more to the wake-up delay than they save)
    __builtin_amdgcn_s_sleep(4);
    // reload every word of the lane (no per-word branches): simple code, few live masks
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int c = tid + BS * k;
#pragma unroll
      for (int q = 0; q < NW; ++q) w[k][q] = (c < L) ? ll_load_word(buf + (long)c * NW + q) : dummy;
    }
    if ((++spins & 255u) == 0u && (spins > kSpinLimit || err_set(err, etag))) {
      ok = false;
      break;
    }
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if constexpr (NW == 1)
      v[k] = ll_value_f(w[k][0]);
    else
      v[k] = bits_to_double(ll_bits64(w[k][0], w[k][1]));
  }
  return ok;
}

// Poll the 2-word FP64 norm partials of all workgroups; lane t reduces entries t + BS*i,
// which all carry the same norm index t % 8.
__device__ __forceinline__ bool gather_norms(const uint64_t* buf, int count, uint32_t tag, uint64_t& mx,
                                             const unsigned* err, uint32_t etag) {
  // count <= 8 * 256 (one entry per workgroup and norm), so a lane has at most two entries
  const int tid = threadIdx.x;
  const int e0 = tid, e1 = tid + BS;
  const uint64_t dummy = (uint64_t)tag << 32;
  uint64_t w0 = e0 < count ? ll_load_word(buf + 2L * e0) : dummy;
  uint64_t w1 = e0 < count ? ll_load_word(buf + 2L * e0 + 1) : dummy;
  uint64_t w2 = e1 < count ? ll_load_word(buf + 2L * e1) : dummy;
  uint64_t w3 = e1 < count ? ll_load_word(buf + 2L * e1 + 1) : dummy;
  unsigned spins = 0;
  bool ok = true;
  while (ll_tag(w0) != tag || ll_tag(w1) != tag || ll_tag(w2) != tag || ll_tag(w3) != tag) {
    __builtin_amdgcn_s_sleep(4);  // as in gather
    w0 = e0 < count ? ll_load_word(buf + 2L * e0) : dummy;
    w1 = e0 < count ? ll_load_word(buf + 2L * e0 + 1) : dummy;
    w2 = e1 < count ? ll_load_word(buf + 2L * e1) : dummy;
    w3 = e1 < count ? ll_load_word(buf + 2L * e1 + 1) : dummy;
    if ((++spins & 255u) == 0u && (spins > kSpinLimit || err_set(err, etag))) {
      ok = false;
      break;
    }
  }
  const uint64_t v0 = e0 < count ? ll_bits64(w0, w1) : 0, v1 = e1 < count ? ll_bits64(w2, w3) : 0;
  mx = v0 > v1 ? v0 : v1;
  return ok;
}

// Poll one FP64 value (two words) until both tags equal `tag`.
__device__ __forceinline__ bool wait_f64(const uint64_t* p, uint32_t tag, double& v, const unsigned* err,
                                         uint32_t etag) {
  uint64_t w0 = ll_load_word(p), w1 = ll_load_word(p + 1);
  unsigned spins = 0;
  bool ok = true;
  while (ll_tag(w0) != tag || ll_tag(w1) != tag) {
    w0 = ll_load_word(p);
    w1 = ll_load_word(p + 1);
    if ((++spins & 255u) == 0u && (spins > kSpinLimit || err_set(err, etag))) {
      ok = false;
      break;
    }
  }
  v = bits_to_double(ll_bits64(w0, w1));
  return ok;
}

// Closed loop: the plant state after solve sv - 1, x_sv = Ad x_{sv-1} + Bd u_{sv-1}. Each
// workgroup keeps its own copy of the state in xpl (parity sv & 1); u comes from the words the
// first nu constraint-row owners published at the end of solve sv - 1 (tag utag), staged in
// ucur. Each wave forms kPlantRows state entries per pass (their loads in flight together):
// per entry, lane-strided FP64 products then a butterfly sum, the same order in every
// workgroup, so every copy is the same. Returns false if the wait for u timed out.
constexpr int kPlantRows = 4;
template <int NWV>
__device__ __forceinline__ bool plant_step(const LayerArgs& a, int sv, uint32_t utag, double* ucur, int* flag) {
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const uint64_t* uw = a.xu + (long)((sv - 1) & 1) * a.nu * 2;
  if (tid < a.nu) {
    double v;
    if (!wait_f64(uw + 2L * tid, utag, v, a.err, utag)) *flag = 1;
    ucur[tid] = v;
  }
  __syncthreads();
  if (*flag) return false;
  const double* xc = a.xpl + ((long)((sv - 1) & 1) * gridDim.x + blockIdx.x) * kMaxPlant;
  double* xn = a.xpl + ((long)(sv & 1) * gridDim.x + blockIdx.x) * kMaxPlant;
  const int nx = a.nx, nu = a.nu;
  for (int rb = wave * kPlantRows; rb < nx; rb += NWV * kPlantRows) {
    double dv[kPlantRows];
    int rc[kPlantRows];  // a valid row index for every slot (entries past nx are not stored)
#pragma unroll
    for (int b = 0; b < kPlantRows; ++b) {
      dv[b] = 0.0;
      rc[b] = rb + b < nx ? rb + b : nx - 1;
    }
    for (int c = lane; c < nx; c += kWave) {
      const double xv = xc[c];
#pragma unroll
      for (int b = 0; b < kPlantRows; ++b) dv[b] = fma(a.Ad[(long)rc[b] * nx + c], xv, dv[b]);
    }
    for (int c = lane; c < nu; c += kWave) {
      const double uv = ucur[c];
#pragma unroll
      for (int b = 0; b < kPlantRows; ++b) dv[b] = fma(a.Bd[(long)rc[b] * nu + c], uv, dv[b]);
    }
#pragma unroll
    for (int b = 0; b < kPlantRows; ++b) {
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) dv[b] += __shfl_xor(dv[b], off, kWave);
      if (lane == 0 && rb + b < nx) xn[rb + b] = dv[b];
    }
  }
  __syncthreads();
  return true;
}

template <typename T, int NC>
struct Cols {
  T v[NC];
};

// Per-thread view of the row it owns (thread tid owns row r0 + tid of the block).
template <typename T>
struct RowState {
  T sx, sz, sy, sq;
  double ax;  // constraint rows, closed loops and scaled problems: (A x)_i carried along
  int R;
  bool own, xrow;
};

// Four consecutive entries of a row of the check matrix (16-byte aligned: ldw is a multiple
// of 4) and of the staged check vector.
__device__ __forceinline__ void load_quad(const float* p, float (&v)[4]) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  v[0] = t.x;
  v[1] = t.y;
  v[2] = t.z;
  v[3] = t.w;
}
__device__ __forceinline__ void load_quad(const double* p, double (&v)[4]) {
  const double2 t0 = *reinterpret_cast<const double2*>(p), t1 = *reinterpret_cast<const double2*>(p + 2);
  v[0] = t0.x;
  v[1] = t0.y;
  v[2] = t1.x;
  v[3] = t1.y;
}

// The residual check's unit of work (an item) is one row of the check matrix over QW = 4 kWave
// check_quads() columns (1024 FP32 / 512 FP64): each lane loads check_quads() quads of it with
// 16-byte loads (16 registers of loads in flight; more raise the kernel's register pressure
// enough to spill loop-invariant values of the iteration loop).
template <typename T>
constexpr int check_quads() {
  return sizeof(T) == sizeof(float) ? 4 : 2;
}
template <typename T>
constexpr int check_width() {
  return 4 * kWave * check_quads<T>();
}
// Items per round of the check: one per wave.
constexpr int kCheckItems = NWAVE;

// The rows of the residual check: dual rows cb .. cb + nck - 1 (x rows of [P, A'], all L
// columns) and primal rows pb .. pb + np - 1 (constraint rows, [A, 0]: the first n columns),
// times [x; y] (cv: this lane's gathered columns tid + BS k). The vector is staged in LDS
// (stage, ch columns at a time: the whole vector when the launch has room for it). The rows of
// a chunk are cut into items (a row over check_width() columns), and every wave takes one item
// per round, so the loads of a whole round are in flight together and no wave waits on a long
// row. Each item leaves its partial sums in LDS, and after every round one thread per row adds
// its row's partials in item order, so the sums do not depend on timing. Row i of the list (dual
// rows first) leaves in res[i]: the product with the x part (P x, or A x) and with the y part
// (A'y; zero for a primal row), both with FP64 accumulation of the exact FP64 products, and
// (FP32 only) the sum of the absolute values of the products, accumulated in FP32 (it only
// enters the rounding bound). Every thread of the workgroup must call it.
template <typename T, int NC>
__device__ __forceinline__ void check_rows(const LayerArgs& a, int cb, int nck, int pb, int np,
                                           const Cols<T, NC>& cv, double (*res)[3], T* stage, int ch) {
  constexpr bool F32 = sizeof(T) == sizeof(float);
  constexpr int QL = check_quads<T>(), QW = check_width<T>();
  __shared__ double part[kCheckItems][3];
  const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int n = a.n, L = a.L;
  const long ldw = a.ldw;
  const T* Cm = static_cast<const T*>(a.C);
  const int rows = nck + np;
  for (int i = tid; i < 3 * rows; i += BS) res[i / 3][i % 3] = 0.0;
  for (int c0 = 0; c0 < L; c0 += ch) {
    __syncthreads();  // the previous chunk has been read (and res cleared)
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int c = tid + BS * k;
      if (c >= c0 && c < c0 + ch) stage[c - c0] = c < L ? cv.v[k] : (T)0;
    }
    // columns of the chunk past L are staged as zero
    if (c0 + ch > L)
      for (int c = L - c0 + tid; c < ch; c += BS) stage[c] = (T)0;
    __syncthreads();
    // items of the chunk: dual rows have pd of them, primal rows pp (columns below n only)
    const int span = L - c0 < ch ? L - c0 : ch;
    const int pd = (span + QW - 1) / QW;
    const int spp = n - c0 < ch ? n - c0 : ch;
    const int pp = spp > 0 ? (spp + QW - 1) / QW : 0;
    const int total = nck * pd + np * pp;
    for (int t0 = 0; t0 < total; t0 += kCheckItems) {
      const int t = t0 + wave;
      if (t < total) {
        const bool dual = t < nck * pd;
        const int i = dual ? t / pd : nck + (t - nck * pd) / pp;
        const int q = dual ? t % pd : (t - nck * pd) % pp;
        const int R = dual ? cb + i : pb + (i - nck);
        const int cl = dual ? L : n;  // columns of this row in the check
        const int cs = c0 + q * QW;  // first column of the item
        const T* row = Cm + (long)R * ldw + cs;
        T w[QL][4];
#pragma unroll
        for (int u = 0; u < QL; ++u) {
          const int cq = 4 * (lane + kWave * u);
          if (cs + cq < cl) {
            load_quad(row + cq, w[u]);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) w[u][e] = (T)0;
          }
        }
        double p = 0.0, q2 = 0.0;
        float fa = 0.0f;
#pragma unroll
        for (int u = 0; u < QL; ++u) {
          const int cq = 4 * (lane + kWave * u);
          T v[4];
          load_quad(stage + q * QW + cq, v);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int c = cs + cq + e;
            const double prod = c < cl ? (double)w[u][e] * (double)v[e] : 0.0;
            if (c < n)
              p += prod;
            else
              q2 += prod;
            if constexpr (F32) fa += c < cl ? fabsf(w[u][e] * v[e]) : 0.0f;
          }
        }
        p = wave_sum_to_last(p);
        q2 = wave_sum_to_last(q2);
        if constexpr (F32) fa = wave_sum_to_last(fa);
        if (lane == kLastLane) {
          part[wave][0] = p;
          part[wave][1] = q2;
          part[wave][2] = (double)fa;
        }
      }
      __syncthreads();
      // one thread per row adds the round's items of its row, in item order
      if (tid < rows) {
        const int lo = tid < nck ? tid * pd : nck * pd + (tid - nck) * pp;
        const int hi = lo + (tid < nck ? pd : pp);
        for (int u = lo > t0 ? lo : t0; u < hi && u < t0 + kCheckItems && u < total; ++u) {
          res[tid][0] += part[u - t0][0];
          res[tid][1] += part[u - t0][1];
          res[tid][2] += part[u - t0][2];
        }
      }
      __syncthreads();
    }
  }
}

// Bound factor of the check in FP32: with the stored matrices and the returned x, z, y rounded
// to FP32 (unit roundoff u = 2^-24), the products exact in FP64 and FP64 accumulation over at
// most L terms here and in the CPU's evaluation, |computed - FP64 value| <= kappa0 * sum |a v|
// per row with kappa0 = 2u + 2 (L + 8) 2^-53; the sum of absolute values is itself accumulated
// in FP32 (relative error below 1e-3 for L <= 8192), hence the factor 1.02. FP64 handles
// compute the FP64 residual itself (0).
template <typename T>
__device__ __forceinline__ double check_kappa(int L) {
  if constexpr (sizeof(T) == sizeof(double)) {
    return 0.0;
  } else {
    return 1.02 * (2.0 * 0x1p-24 + 2.0 * (double)(L + 8) * 0x1p-53);
  }
}
template <typename T>
__device__ __forceinline__ double unit_roundoff() {
  return sizeof(T) == sizeof(double) ? 0.0 : 1.01 * 0x1p-24;
}

struct CheckOut {
  int status;  // ST_* (ST_RUNNING: continue)
  int jn;      // grid index for the next iterations
  bool ok;     // false: an exchange timed out
};

// Residual check (eqs. primal, dual), stopping test and penalty rule (eq. rho_update; nearest
// grid value, Sec. III-C) at iteration k, check number nchk, in two halves so that the caller
// can reload its register rows while the norms are exchanged. Every workgroup takes the same
// decision.
//
// check_partials: [x; y] to every workgroup; dual side: this workgroup's share of the x rows of
// [P, A'] [x; y]; primal side: A x for the constraint rows it owns, formed afresh from the
// check matrix (FP64 accumulation); the seven partial inf-norms published. With the iteration
// in FP32 the published r_p and r_d are upper bounds, and ||Ax||, ||z||, ||Px||, ||A'y||,
// ||q|| lower bounds, of the FP64 values a CPU evaluation of the returned x, z, y with the
// caller's FP64 P, q, A gives (check_kappa), so SOLVED implies that the FP64 test passes. The
// owner of a constraint row gets its fresh (A x)_i in ax_out. Returns false if an exchange
// timed out.
template <typename T, int NC, bool XT>
__device__ __forceinline__ bool check_partials(const LayerArgs& a, const RowState<T>& rs, int r0, int nrows,
                                               int cb, int nck, const T* cq, int k, int nchk, uint32_t tag,
                                               double (*res)[3], T* stage, double& ax_out) {
  __shared__ unsigned long long nmax[8];  // the workgroup's partial norms (ordered bit patterns)
  constexpr int NW = LLWords<T>::kWords;
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int L = a.L;
  if (tid < 8) nmax[tid] = 0ull;  // ordered before the atomics below by check_rows' barriers

  // [x; y] to every workgroup
  const uint32_t ctag = tag + (uint32_t)k;
  uint64_t* xc = a.xc + (long)(nchk & 1) * L * NW;
  if (rs.own) ll_store(xc + (long)rs.R * NW, rs.xrow ? rs.sx : rs.sy, ctag);
  Cols<T, NC> cv;
  const bool ok2 = gather<T, NC>(xc, L, ctag, cv.v, a.err, tag);
  if (__syncthreads_or(!ok2)) return false;
  const double kappa = check_kappa<T>(L), ut = unit_roundoff<T>();
  uint64_t nb[7] = {0, 0, 0, 0, 0, 0, 0};
  // dual side: rows cb .. cb + nck - 1 of [P, A'] [x; y]; primal side: the constraint rows
  // this workgroup owns, [A, 0] [x; y]
  const int pb = r0 > a.n ? r0 : a.n;
  const int np = r0 + nrows > pb ? r0 + nrows - pb : 0;
  check_rows<T, NC>(a, cb, nck, pb, np, cv, res, stage, a.check_cols);
  if (tid < nck) {
    const double pr = res[tid][0], ar = res[tid][1], d = kappa * res[tid][2];
    const double qv = (double)cq[tid], dq = ut * fabs(qv);
    const double f = XT && a.sc_dual ? a.sc_dual[cb + tid] : 1.0;  // original units
    nb[N_RD] = abs_bits(f * (fabs(pr + qv + ar) + d + dq));
    nb[N_PX] = abs_bits(f * lower_bound(fabs(pr), d));
    nb[N_ATY] = abs_bits(f * lower_bound(fabs(ar), d));
    nb[N_Q] = abs_bits(f * lower_bound(fabs(qv), dq));
  }
  if (rs.own && !rs.xrow) {
    const int i = nck + rs.R - pb;
    const double s = res[i][0], ds = kappa * res[i][2];
    const double zv = (double)rs.sz, dz = ut * fabs(zv);
    const double e = XT && a.sc_prim ? a.sc_prim[rs.R - a.n] : 1.0;
    nb[N_RP] = abs_bits(e * (fabs(s - zv) + ds + dz));
    nb[N_AX] = abs_bits(e * lower_bound(fabs(s), ds));
    nb[N_Z] = abs_bits(e * lower_bound(fabs(zv), dz));
    ax_out = s;
  }
  // only the threads of the check and constraint rows hold values: LDS atomics, no wave-wide
  // reductions
#pragma unroll
  for (int i = 0; i < 7; ++i)
    if (nb[i]) atomicMax(&nmax[i], (unsigned long long)nb[i]);
  __syncthreads();
  if (tid < 8) {
    uint64_t v = 0;
    if (tid < 7) {
      v = nmax[tid];
    } else {
      // the host-mapped flag costs a PCIe round trip (~13 us measured), so it is read at
      // every kAbortEvery-th check only
      const bool ab = (nchk % kAbortEvery) == kAbortEvery - 1 && a.abort_flag &&
                      __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      v = err_set(a.err, tag) ? 2u : (ab ? 1u : 0u);
    }
    ll_store_bits64(a.xn + ((long)(nchk & 1) * G * 8 + (long)g * 8 + tid) * 2, v, ctag);
  }
  return true;
}

// check_decide: every workgroup reads all partial norms, evaluates the stopping test and the
// penalty rule, and records the check (workgroup 0).
template <typename T>
__device__ __forceinline__ CheckOut check_decide(const LayerArgs& a, const RhoTable& rt, int k, int nchk, int j,
                                                 uint32_t tag, long hoff) {
  __shared__ uint64_t nred[NWAVE][8];
  __shared__ uint64_t nfin[8];
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid % kWave, wave = tid / kWave;
  const uint32_t ctag = tag + (uint32_t)k;
  CheckOut out{ST_RUNNING, j, true};
  uint64_t mx;
  const bool ok3 = gather_norms(a.xn + (long)(nchk & 1) * G * 8 * 2, G * 8, ctag, mx, a.err, tag);
  // lanes with equal tid % 8 hold the same norm index
#pragma unroll
  for (int off = 8; off < kWave; off <<= 1) {
    const uint64_t o = __shfl_xor(mx, off, kWave);
    mx = o > mx ? o : mx;
  }
  if (lane < 8) nred[wave][lane] = mx;
  if (__syncthreads_or(!ok3)) {
    out.ok = false;
    return out;
  }
  if (tid < 8) {
    uint64_t v = 0;
    for (int w = 0; w < NWAVE; ++w) v = nred[w][tid] > v ? nred[w][tid] : v;
    nfin[tid] = v;
  }
  __syncthreads();

  // one thread decides (every workgroup sees the same bits, so all decide alike) and the
  // workgroup reads the decision back from LDS
  __shared__ int decision[2];
  if (tid == 0) {
    bool nonfinite = false;
#pragma unroll
    for (int i = 0; i < 7; ++i) nonfinite |= nfin[i] >= kInfBits;
    const double rp = bits_to_double(nfin[N_RP]), rd = bits_to_double(nfin[N_RD]);
    const double nax = bits_to_double(nfin[N_AX]), nz = bits_to_double(nfin[N_Z]);
    const double npx = bits_to_double(nfin[N_PX]), naty = bits_to_double(nfin[N_ATY]);
    const double nq = bits_to_double(nfin[N_Q]);
    const uint64_t flags = nfin[N_FLAGS];
    int st = ST_RUNNING;
    if (nonfinite) {
      st = ST_NONFINITE;
    } else if (a.terminate) {
      const double eps_p = a.eps_abs + a.eps_rel * fmax(nax, nz);
      const double eps_d = a.eps_abs + a.eps_rel * fmax(fmax(npx, naty), nq);
      if (rp <= eps_p && rd <= eps_d) st = ST_SOLVED;
    }
    if (st == ST_RUNNING && k == a.max_iter) st = ST_MAX_ITER;
    if (st == ST_RUNNING && flags >= 2) st = ST_INTERNAL;
    if (st == ST_RUNNING && flags == 1) st = ST_ABORTED;
    int jn = j;
    if (st == ST_RUNNING && a.n_rho > 1 && rp > 0.0 && rd > 0.0) {
      const double num = rp * fmax(fmax(npx, naty), fmax(nq, 1e-4));
      const double den = rd * fmax(fmax(nax, nz), 1e-4);
      const double rh = rt.grid[j] * sqrt(num / den);
      jn = 0;
      while (jn < a.n_rho - 1 && rh > rt.mid[jn]) ++jn;
    }
    if (g == 0) {
      if (a.rho_hist) a.rho_hist[hoff + nchk] = jn;
      if (a.prim_res) a.prim_res[hoff + nchk] = rp;
      if (a.dual_res) a.dual_res[hoff + nchk] = rd;
    }
    decision[0] = st;
    decision[1] = jn;
  }
  __syncthreads();
  out.status = decision[0];
  out.jn = decision[1];
  __syncthreads();  // nfin, nred and decision are reused by the next check
  return out;
}

template <typename T, bool XT>
__device__ __forceinline__ void finish(const LayerArgs& a, RowState<T> rs, int sv, int k, int st, int j,
                                       uint32_t tag, const double* exs) {
  if (rs.own) {
    // the handle keeps the (scaled) iterates; the outputs are in original units
    if (rs.xrow) {
      static_cast<T*>(a.xs)[rs.R] = rs.sx;
      static_cast<T*>(a.xo)[(long)sv * a.n + rs.R] = XT && a.un_x ? (T)(a.un_x[rs.R] * (double)rs.sx) : rs.sx;
    } else {
      const int i = rs.R - a.n;
      static_cast<T*>(a.zs)[i] = rs.sz;
      static_cast<T*>(a.ys)[i] = rs.sy;
      a.axs[i] = rs.ax;
      static_cast<T*>(a.zo)[(long)sv * a.m + i] = XT && a.sc_prim ? (T)(a.sc_prim[i] * (double)rs.sz) : rs.sz;
      static_cast<T*>(a.yo)[(long)sv * a.m + i] = XT && a.un_y ? (T)(a.un_y[i] * (double)rs.sy) : rs.sy;
      if (XT && a.Ad && i < a.nu) {
        // the first stage's applied control (the clamped constraint row plus its E x_s part)
        const double uv = ((double)rs.sz + exs[threadIdx.x]) * (a.sc_prim ? a.sc_prim[i] : 1.0);
        a.traj_u[(long)sv * a.nu + i] = uv;
        ll_store(a.xu + ((long)(sv & 1) * a.nu + i) * 2, uv, tag);
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.iterations[sv] = k;
    a.status[sv] = st;
    a.rho_index[sv] = j;
    *a.js = j;
  }
}

template <typename T, int NC, int NRS>
__device__ __forceinline__ void load_stationary(const LayerArgs& a, int j, int r0, int nstat, T (&wst)[NRS][NC]) {
  const T* Wj = static_cast<const T*>(a.W) + (long)j * a.w_stride;
  const int tid = threadIdx.x;
#pragma unroll
  for (int rr = 0; rr < NRS; ++rr)
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int c = tid + BS * k;
      wst[rr][k] = (rr < nstat && c < a.L) ? Wj[(long)(r0 + rr) * a.ldw + c] : (T)0;
    }
}

// Rows NRS .. NRS + NLM - 1 of the block live in LDS for the whole solve, laid out
// [row][k][lane] so that every lane reads and writes only its own words (no barrier needed,
// no bank conflicts). Rows past the end of the block are zero, so the row loops need no
// per-row branches.
template <typename T, int NC, int NLM>
__device__ __forceinline__ void load_lds_rows(const LayerArgs& a, int j, int r0, int first, int nlds, T* wl) {
  const T* Wj = static_cast<const T*>(a.W) + (long)j * a.w_stride;
  const int tid = threadIdx.x;
  // batches of RB rows: their loads first (branch-free: masked entries read a valid address),
  // then the LDS stores
  constexpr int RB = 16 / NC < 1 ? 1 : (16 / NC > NLM ? NLM : 16 / NC);
#pragma unroll 1
  for (int r0b = 0; r0b < NLM; r0b += RB) {
    T v[RB][NC];
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const int rr = r0b + b, c = tid + BS * k;
        v[b][k] = Wj[(rr < nlds && c < a.L) ? (long)(r0 + first + rr) * a.ldw + c : 0];
      }
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const int rr = r0b + b, c = tid + BS * k;
        if (rr < NLM) wl[(rr * NC + k) * BS + tid] = (rr < nlds && c < a.L) ? v[b][k] : (T)0;
      }
  }
}

// NRS rows of each block in registers, NLM in LDS, the rest streamed. The loop between two
// checks is kept free of everything the check needs, and the register rows are reloaded at
// every check, so the check code does not compete with them for registers.
// The kernel reads its arguments through the kernarg segment pointer made opaque at the start of
// each phase (fresh), so a phase loads the fields it uses instead of every field of the whole
// persistent loop staying in scalar registers (which spills them into vector registers).
typedef const __attribute__((address_space(4))) LayerArgs* cargs_t;
__device__ __forceinline__ const LayerArgs& fresh(cargs_t p) {
  asm volatile("" : "+s"(p));
  return *(const LayerArgs*)p;
}

template <typename T, int NC, int NRS, int NLM, bool XT>
__global__ void __launch_bounds__(BS) layer_kernel(LayerArgs a_in) {
  (void)a_in;
  const cargs_t kp = (cargs_t)__builtin_amdgcn_kernarg_segment_ptr();
  const LayerArgs& a = fresh(kp);
  constexpr int NW = LLWords<T>::kWords;
  __shared__ T red[NWAVE][kMaxRows];
  __shared__ int fail_flag;
  __shared__ RhoTable rt;
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  T* wl = reinterpret_cast<T*>(dyn_lds);
  T* const cstage = wl + NLM * NC * BS;  // the check vector (check_cols entries) after the LDS rows

  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid % kWave, wave = tid / kWave;
  const int n = a.n, L = a.L;
  const int rbase = L / G, rextra = L % G;
  const int nrows = rbase + (g < rextra ? 1 : 0);
  const int r0 = g * rbase + (g < rextra ? g : rextra);
  const int nstat = nrows < NRS ? nrows : NRS;
  const int nlds = nrows - nstat < NLM ? nrows - nstat : NLM;
  constexpr int nres = NRS + NLM;  // rows held on chip; rows nres..nrows-1 stream from memory
  constexpr int RON = NRS + NLM;
  const int my_row = rows_held<RON>();
  const bool writer = row_writer<RON>();
  if (tid == 0) fail_flag = 0;
  if (tid < a.n_rho) rt.grid[tid] = a.grid[tid];
  if (tid < a.n_rho - 1) rt.mid[tid] = a.mid[tid];
  __syncthreads();

  // Solves s = 0 .. count-1 run one after another in this launch; the weights of the active
  // penalty stay on chip between them. Solve s uses tags tag0 + s * span, takes its data from
  // x0 + s * nx (when given) and writes its results at index s of the outputs.
  const uint32_t span = (uint32_t)a.max_iter + 2u;
  const int ci = a.check_interval, max_iter = a.max_iter;
  RowState<T> rs;
  rs.own = tid < nrows;
  rs.R = r0 + tid;
  rs.xrow = rs.R < n;
  rs.sx = rs.sz = rs.sy = rs.sq = (T)0;
  rs.ax = 0.0;
  T sl = 0, su = 0;
  bool seq = false;
  if (rs.own && !rs.xrow) seq = a.eq[rs.R - n] != 0;
  int j = a.warm ? *a.js : a.j0;
  int lds_j = -1;  // penalty index of the rows now in LDS
  int wst_j = -1;  // penalty index of the rows now in registers
  T wst[NRS][NC];
  __shared__ T upd[kMaxRows][2];
  // this workgroup's share of the x rows for the dual side of the check, and their q
  // (split_term, split_row: a running maximum over h <= g, here a prefix maximum over wave 0,
  // lane l holding h = 4 l + 1 .. 4 l + 4; the grid has at most 256 workgroups)
  __shared__ int split[2];
  if (wave == 0) {
    double run = 0.0, mh[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 4 * lane + i + 1;
      const double f = h <= G ? split_term(h, G, n, a.m, L) : 0.0;
      run = f > run ? f : run;
      mh[i] = run;
    }
    double inc = run;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const double o = __shfl_up(inc, off, kWave);
      if (lane >= off) inc = o > inc ? o : inc;
    }
    double exc = __shfl_up(inc, 1, kWave);
    if (lane == 0) exc = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 4 * lane + i + 1;
      const double best = exc > mh[i] ? exc : mh[i];
      if (h == g) split[0] = split_row(best, n, L);
      if (h == g + 1) split[1] = split_row(best, n, L);
    }
    if (g == 0 && lane == 0) split[0] = 0;
  }
  __syncthreads();
  const int cb = split[0], nck = split[1] - split[0];
  __shared__ T cq[kMaxCheckRows];
  __shared__ double cres[kMaxCheckRows + kMaxRows][3];  // check_rows results: dual, then primal rows
  // closed loop: (E x_s)_i of the owned constraint rows; the applied control
  __shared__ double exs[kMaxRows];
  __shared__ double ucur[kMaxPlant];
  // XT instantiations also run closed loops and scaled problems; the others carry none of
  // that code (its registers would cost the plain solves)
  const bool closed = XT && a.Ad != nullptr;

  for (int sv = 0; sv < a.count; ++sv) {
    const LayerArgs& a = fresh(kp);
    const uint32_t tag = a.tag + (uint32_t)sv * span;
    const bool warm = sv == 0 ? a.warm != 0 : a.chain != 0;

    // update from an initial state (Sec. IV): q = F x0 for x rows, l = lo - E x0 and
    // u = hi - E x0 for constraint rows, FP64 products, one wave per row of the block; the
    // values reach the owners through LDS and are written back for later solves
    __syncthreads();  // upd[] and cq[] of the previous solve have been read
    double* xpl = closed ? a.xpl + ((long)(sv & 1) * G + g) * kMaxPlant : nullptr;
    if (closed) {
      if (sv == 0) {
        for (int c = tid; c < a.nx; c += BS) xpl[c] = a.x0[c];
        __syncthreads();
      } else if (!plant_step<NWAVE>(a, sv, tag - span, ucur, &fail_flag)) {
        if (tid == 0) err_raise(a.err, tag);
        finish<T, XT>(a, rs, sv, 0, ST_INTERNAL, j, tag, exs);
        return;
      }
      if (g == 0)
        for (int c = tid; c < a.nx; c += BS) a.traj_x[(long)sv * a.nx + c] = xpl[c];
    }
    if (a.x0) {
      const double* x0 = closed ? xpl : a.x0 + (long)sv * a.nx;
      // rows 0 .. nrows-1: owned layer rows; rows nrows .. nrows+nck-1: the check's x rows
      for (int rr = wave; rr < nrows + nck; rr += NWAVE) {
        const int R = rr < nrows ? r0 + rr : cb + (rr - nrows);
        const double* arow = R < n ? a.F + (long)R * a.nx : a.E + (long)(R - n) * a.nx;
        double dv = 0.0;
        for (int c = lane; c < a.nx; c += kWave) dv = fma(arow[c], x0[c], dv);
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) dv += __shfl_xor(dv, off, kWave);
        if (lane == 0) {
          if (rr >= nrows) {
            cq[rr - nrows] = (T)dv;
          } else if (R < n) {
            upd[rr][0] = (T)dv;
            static_cast<T*>(const_cast<void*>(a.q))[R] = (T)dv;
          } else {
            const int i = R - n;
            if constexpr (XT) exs[rr] = dv;
            upd[rr][0] = (T)(a.plo[i] - dv);
            upd[rr][1] = (T)(a.phi[i] - dv);
            static_cast<T*>(const_cast<void*>(a.l))[i] = upd[rr][0];
            static_cast<T*>(const_cast<void*>(a.u))[i] = upd[rr][1];
          }
        }
      }
    } else if (tid < nck) {
      cq[tid] = static_cast<const T*>(a.q)[cb + tid];
    }
    __syncthreads();

    // row-owner state: cold (zero, start penalty), warm from the handle (first solve) or from
    // the previous solve of this launch. In the XT instantiation (closed loops, scaled
    // problems) a warm start that continues a solve takes z = A x from the product the
    // constraint-row owners carried along it (in registers within the launch, from the
    // handle's copy across launches); otherwise, and for a caller-given x, z = A x is formed
    // through the check product (keeping the carried value live costs the plain loop).
    const bool carried = XT && warm && (sv > 0 || a.warm_ax != 0);
    if (rs.own) {
      if (rs.xrow) {
        rs.sq = a.x0 ? upd[tid][0] : static_cast<const T*>(a.q)[rs.R];
        if (!warm) rs.sx = (T)0;
        else if (sv == 0) rs.sx = static_cast<const T*>(a.xs)[rs.R];
      } else {
        const int i = rs.R - n;
        sl = a.x0 ? upd[tid][0] : static_cast<const T*>(a.l)[i];
        su = a.x0 ? upd[tid][1] : static_cast<const T*>(a.u)[i];
        if (!warm) rs.sy = (T)0;
        else if (sv == 0) rs.sy = static_cast<const T*>(a.ys)[i];
        if (!carried) rs.ax = 0.0;
        else if (sv == 0) rs.ax = a.axs[i];
        rs.sz = carried ? (T)rs.ax : (T)0;
      }
    }
    if (!warm) j = a.j0;
    T srho = (T)(rt.grid[j] * (seq ? a.rho_eq_scale : 1.0));
    if (j != lds_j) {
      load_lds_rows<T, NC, NLM>(a, j, r0, NRS, nlds, wl);
      lds_j = j;
    }
    __syncthreads();  // fail_flag, LDS rows
    int nchk = 0;

    // warm start from a caller-given x: z = A x (Sec. II-B, warm starting)
    if (warm && !carried) {
      if (rs.own) ll_store(a.xc + (long)rs.R * NW, rs.xrow ? rs.sx : rs.sy, tag);
      Cols<T, NC> cv;
      const bool ok = gather<T, NC>(a.xc, L, tag, cv.v, a.err, tag);
      if (__syncthreads_or(!ok)) {
        if (tid == 0) err_raise(a.err, tag);
        finish<T, XT>(a, rs, sv, 0, ST_INTERNAL, j, tag, exs);
        return;
      }
      // the constraint rows of the block: [A, 0] [x; y]
      const int pb = r0 > n ? r0 : n;
      check_rows<T, NC>(a, 0, 0, pb, r0 + nrows > pb ? r0 + nrows - pb : 0, cv, cres, cstage, a.check_cols);
      if (rs.own && !rs.xrow) {
        rs.ax = cres[rs.R - pb][0];
        rs.sz = (T)rs.ax;
      }
    }

    // first layer input w_1
    {
      const T sigma = (T)a.sigma;
      const T w1 = rs.xrow ? sigma * rs.sx - rs.sq : srho * rs.sz - rs.sy;
      if (rs.own) ll_store(a.xw + ((long)L + rs.R) * NW, w1, tag + 1u);
    }

    // the register rows of the active penalty: loaded at the start unless the previous solve
    // left them in place, and at every check while the norms are exchanged (dead during the
    // check's own work, so they do not compete with it for registers)
    if (wst_j != j) {
      load_stationary<T, NC, NRS>(a, j, r0, nstat, wst);
      wst_j = j;
    }
    int k = 0;
    while (true) {
      const int kend = (k / ci + 1) * ci < max_iter ? (k / ci + 1) * ci : max_iter;
      {
        const LayerArgs& a = fresh(kp);
        const T alpha = (T)a.alpha, oma = (T)(1.0 - a.alpha), sigma = (T)a.sigma;
        [[maybe_unused]] const double alpha_d = a.alpha, oma_d = 1.0 - a.alpha;
        uint64_t* xw = a.xw;
        while (k < kend) {
          ++k;
          // layer matvec: rows of Wc_j times w_k
          T wv[NC];
          const bool ok = gather<T, NC>(xw + (long)(k & 1) * L * NW, L, tag + (uint32_t)k, wv, a.err, tag);
          if (!ok) fail_flag = 1;
          // all on-chip rows, then one multi-row wave reduction (rows past the block are zero)
          T acc[RON];
#pragma unroll
          for (int rr = 0; rr < RON; ++rr) {
            acc[rr] = 0;
            if (rr < NRS) {
#pragma unroll
              for (int k2 = 0; k2 < NC; ++k2) acc[rr] = fma(wst[rr < NRS ? rr : 0][k2], wv[k2], acc[rr]);
            } else {
#pragma unroll
              for (int k2 = 0; k2 < NC; ++k2) acc[rr] = fma(wl[((rr - NRS) * NC + k2) * BS + tid], wv[k2], acc[rr]);
            }
          }
          const T rsum = reduce_rows<RON>(acc);
          if (writer) red[wave][my_row] = rsum;
          if (nrows > nres) {
            const T* Wj = static_cast<const T*>(a.W) + (long)j * a.w_stride;
            for (int rr = nres; rr < nrows; ++rr) {
              T acc1 = 0;
#pragma unroll
              for (int k2 = 0; k2 < NC; ++k2) {
                const int c = tid + BS * k2;
                acc1 = fma(c < L ? Wj[(long)(r0 + rr) * a.ldw + c] : (T)0, wv[k2], acc1);
              }
              acc1 = wave_sum_to_last(acc1);
              if (lane == kLastLane) red[wave][rr] = acc1;
            }
          }
          __syncthreads();
          if (fail_flag) {
            if (tid == 0) err_raise(a.err, tag);
            finish<T, XT>(a, rs, sv, k, ST_INTERNAL, j, tag, exs);
            return;
          }

          // row-local update: relaxation, clamp (eq. clamp), dual update
          if (rs.own) {
            T v = 0;
#pragma unroll
            for (int w = 0; w < NWAVE; ++w) v += red[w][tid];
            if (rs.xrow) {
              rs.sx = alpha * v + oma * rs.sx;
            } else {
              // closed loops, scaled problems: A x_{k+1} = alpha A x~ + (1 - alpha) A x_k, with
              // A x~ the layer output v (the z = A x of a warm start that continues this solve)
              if constexpr (XT) rs.ax = fma(alpha_d, (double)v, oma_d * rs.ax);
              const T t = alpha * v + oma * rs.sz + rs.sy / srho;
              const T zn = box_clamp(t, sl, su);
              rs.sy = srho * (t - zn);
              rs.sz = zn;
            }
            // No barrier after this: a wave passes the next gather only after every row of the
            // block was published, and each owner publishes after it has read red[][].
            if (k < kend) {
              const T wn = rs.xrow ? sigma * rs.sx - rs.sq : srho * rs.sz - rs.sy;
              ll_store(xw + ((long)((k + 1) & 1) * L + rs.R) * NW, wn, tag + (uint32_t)(k + 1));
            }
          }
        }
      }

      const LayerArgs& ac = fresh(kp);
      // a fixed budget that is not a multiple of the check interval ends without a check
      // (closed loops; they run the XT instantiation)
      if constexpr (XT) {
        if (!ac.final_check && k == max_iter && k % ci != 0) {
          finish<T, XT>(ac, rs, sv, k, ST_MAX_ITER, j, tag, exs);
          break;  // next solve of the sequence
        }
      }

      // check at iteration k (every check_interval iterations and at max_iter)
      __syncthreads();
      CheckOut co{ST_RUNNING, j, false};
      if (check_partials<T, NC, XT>(ac, rs, r0, nrows, cb, nck, cq, k, nchk, tag, cres, cstage, rs.ax)) {
        load_stationary<T, NC, NRS>(ac, j, r0, nstat, wst);  // in flight while the norms are exchanged
        wst_j = j;
        co = check_decide<T>(ac, rt, k, nchk, j, tag, (long)sv * ac.max_checks);
      }
      ++nchk;
      if (!co.ok) {
        if (tid == 0) err_raise(ac.err, tag);
        finish<T, XT>(ac, rs, sv, k, ST_INTERNAL, j, tag, exs);
        return;
      }
      if (co.status != ST_RUNNING) {
        finish<T, XT>(ac, rs, sv, k, co.status, j, tag, exs);
        break;  // next solve of the sequence
      }
      if (co.jn != j) {
        j = co.jn;
        srho = (T)(rt.grid[j] * (seq ? ac.rho_eq_scale : 1.0));
        load_lds_rows<T, NC, NLM>(ac, j, r0, NRS, nlds, wl);
        lds_j = j;
        load_stationary<T, NC, NRS>(ac, j, r0, nstat, wst);
        wst_j = j;
      }
      const T sigma = (T)ac.sigma;
      const T wn = rs.xrow ? sigma * rs.sx - rs.sq : srho * rs.sz - rs.sy;
      if (rs.own) ll_store(ac.xw + ((long)((k + 1) & 1) * L + rs.R) * NW, wn, tag + (uint32_t)(k + 1));
    }
  }

  // closed loop: the state after the last control, written by workgroup 0
  if (closed && g == 0) {
    const uint32_t last = a.tag + (uint32_t)(a.count - 1) * span;
    __syncthreads();
    if (!plant_step<NWAVE>(a, a.count, last, ucur, &fail_flag)) {
      if (tid == 0) err_raise(a.err, last);
      return;
    }
    const double* xf = a.xpl + ((long)(a.count & 1) * G + g) * kMaxPlant;
    for (int c = tid; c < a.nx; c += BS) a.traj_x[(long)a.count * a.nx + c] = xf[c];
  }
}

template <typename T>
constexpr int words() {
  return LLWords<T>::kWords;
}

// Register rows: 32 registers of weights per lane; as many LDS rows again, so that the on-chip
// rows are a power of two (the multi-row reduction needs one) and at most 32 (accumulators).
template <typename T, int NC>
constexpr int reg_rows() {
  return 32 / (NC * words<T>()) > 16 / words<T>() ? 16 / words<T>() : 32 / (NC * words<T>());
}
template <typename T, int NC>
constexpr int lds_rows_max() {
  return reg_rows<T, NC>();
}

struct KernelChoice {
  const void* fn;
  int nc, nrs, nlm;
};

template <typename T, int NC>
KernelChoice pick_kernel(bool xt) {
  constexpr int nrs = reg_rows<T, NC>();
  constexpr int nlm = lds_rows_max<T, NC>();
  const void* fn = xt ? reinterpret_cast<const void*>(&layer_kernel<T, NC, nrs, nlm, true>)
                      : reinterpret_cast<const void*>(&layer_kernel<T, NC, nrs, nlm, false>);
  return KernelChoice{fn, NC, nrs, nlm};
}

template <typename T>
KernelChoice kernel_for(int L, bool xt) {
  if (L <= BS) return pick_kernel<T, 1>(xt);
  if (L <= 2 * BS) return pick_kernel<T, 2>(xt);
  if (L <= 4 * BS) return pick_kernel<T, 4>(xt);
  if (L <= 8 * BS) return pick_kernel<T, 8>(xt);
  return KernelChoice{nullptr, 0, 0, 0};
}

}  // namespace

template <typename T>
LaunchPlan plan_layer(int L, int grid, bool xt) {
  LaunchPlan p{};
  const KernelChoice kc = kernel_for<T>(L, xt);
  if (!kc.fn || grid < 1) return p;
  int dev = 0, smem_max = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return p;
  if (hipDeviceGetAttribute(&smem_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return p;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return p;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, kc.fn) != hipSuccess) return p;
  const long row_bytes = (long)kc.nc * BS * sizeof(T);
  const long room = (long)smem_max - (long)fa.sharedSizeBytes;
  const int lds_rows = kc.nlm;  // the kernel always keeps NLM rows (zeros past the block)
  // the check vector takes the rest of LDS, whole if it fits, in multiples of a check item
  const long qw = check_width<T>();
  const long left = room - (long)lds_rows * row_bytes;
  const long whole = ((long)L + qw - 1) / qw * qw;
  long ch = left / (long)sizeof(T) / qw * qw;
  if (ch > whole) ch = whole;
  if (ch < qw) return p;
  p.fn = kc.fn;
  p.lds_rows = lds_rows;
  p.check_cols = (int)ch;
  p.dyn_bytes = (size_t)lds_rows * row_bytes + (size_t)ch * sizeof(T);
  if (hipFuncSetAttribute(kc.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.dyn_bytes) != hipSuccess) {
    p.fn = nullptr;
    return p;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kc.fn, BS, p.dyn_bytes) != hipSuccess) {
    p.fn = nullptr;
    return p;
  }
  p.max_grid = per_cu * cus;
  p.reg_rows = kc.nrs;
  return p;
}

template <typename T>
hipError_t launch_layer(const LayerArgs& a, const LaunchPlan& p, int grid, hipStream_t st) {
  if (!p.fn) return hipErrorInvalidValue;
  LayerArgs copy = a;
  copy.lds_rows = p.lds_rows;
  copy.check_cols = p.check_cols;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(p.fn, dim3(grid), dim3(BS), args, p.dyn_bytes, st);
}

template LaunchPlan plan_layer<float>(int, int, bool);
template LaunchPlan plan_layer<double>(int, int, bool);
template hipError_t launch_layer<float>(const LayerArgs&, const LaunchPlan&, int, hipStream_t);
template hipError_t launch_layer<double>(const LayerArgs&, const LaunchPlan&, int, hipStream_t);

}  // namespace rqp
