// Device engine for gfx950: device tables, the matrix-vector product
// kernels of the MLFMA (Sec. IV) and the GMRES driver (Sec. V stage v).
//
// Data layout in HBM (box-major, sample-contiguous):
//   x, y        [R][P][n]            n = 2N unknowns per particle
//   S_l, G_l    [R][box_l][2][K_l]   outgoing / incoming transverse pattern
//                                     (theta, phi components) per box;
//                                     sample s = it * np + ip
//   TL_l        [49][K_l]            translation function per box offset
// Every kernel writes each output element once (no atomics), so repeated
// products are bitwise reproducible.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>
#include <cstdint>
#include <chrono>
#include <cxxabi.h>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "engine.hpp"

namespace mlfma {

namespace {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
  T x, y;
};
// two complex values loaded together (one 16-byte load in FP32)
template <typename T>
struct alignas(4 * sizeof(T)) CP {
  C2<T> a, b;
};

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc += a b as four chained fused multiply-adds (one rounding each)
template <typename T>
__device__ __forceinline__ void cfma(C2<T>& acc, C2<T> a, C2<T> b) {
  acc.x = fmadd(a.x, b.x, acc.x);
  acc.x = fmadd(-a.y, b.y, acc.x);
  acc.y = fmadd(a.x, b.y, acc.y);
  acc.y = fmadd(a.y, b.x, acc.y);
}
template <typename T>
__device__ __forceinline__ void cfma_conj_a(C2<T>& acc, C2<T> a, C2<T> b) {  // acc += conj(a) b
  acc.x = fmadd(a.x, b.x, acc.x);
  acc.x = fmadd(a.y, b.y, acc.x);
  acc.y = fmadd(a.x, b.y, acc.y);
  acc.y = fmadd(-a.y, b.x, acc.y);
}
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C2<T> cmul_conj_a(C2<T> a, C2<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
// Element i of the array at p, its byte offset formed in 32 bits: with p
// uniform over the wave the access takes the scalar-base form of a global
// load or store (one shift per access instead of a 64-bit address sum).
// The caller guarantees i * sizeof(U) < 2^32.
template <typename U>
__device__ __forceinline__ U& at32(U* p, unsigned i) {
  using B = typename std::conditional<std::is_const<U>::value, const char, char>::type;
  return *reinterpret_cast<U*>(reinterpret_cast<B*>(p) + i * (unsigned)sizeof(U));
}

// Short symbol of a kernel (name and template arguments, without namespace,
// return type or parameter list), as the runtime names it: the unit in
// which kernel traces report.
inline std::string kernel_symbol(const void* fn, hipStream_t st) {
  const char* m = hipKernelNameRefByPtr(fn, st);
  if (!m) return std::string();
  int status = 0;
  char* d = abi::__cxa_demangle(m, nullptr, nullptr, &status);
  std::string n = (status == 0 && d) ? std::string(d) : std::string(m);
  std::free(d);
  for (const char* pre : {"void ", "mlfma::", "(anonymous namespace)::"}) {
    size_t at;
    while ((at = n.find(pre)) != std::string::npos) n.erase(at, std::strlen(pre));
  }
  // cut the parameter list: the first '(' outside template brackets
  int depth = 0;
  for (size_t i = 0; i < n.size(); ++i) {
    if (n[i] == '<') ++depth;
    else if (n[i] == '>') --depth;
    else if (n[i] == '(' && depth == 0) return n.substr(0, i);
  }
  return n;
}

constexpr int kBlock = 256;

// Static device scratch of the no-allocation product (mlfma_matvec_noalloc):
// its pattern buffers live here instead of in context allocations.  Every
// GPU the library runs on holds one copy until the process ends; calls on one
// GPU share it and keep the last call's contents.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current (the array's name in host code is not a
// device address).
int scratch_address(void** out, std::string& err) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    err = std::string("hipGetDevice failed: ") + hipGetErrorString(e);
    return -3;
  }
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      return -3;
    }
    it = addr.emplace(dev, p).first;
  }
  *out = it->second;
  return 0;
}


#define HIP_TRY(expr)                                                     \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      err = std::string(#expr " failed: ") + hipGetErrorString(e_);       \
      return -3;                                                          \
    }                                                                     \
  } while (0)

// ------------------------------------------------------------ near field --
// y[r][p] = sum over the neighbour slots o of M_{slot(p,o)} x[r][nbr(p,o)].
// A block handles TPN consecutive particles (4 waves x PW particles; lane =
// output row, rows lane and lane + 64).  For each slot o the x vectors of
// the tile's o-neighbours are staged in LDS; when every particle of the tile
// that has an o-neighbour uses the same matrix (tile_slot >= 0) the matrix
// is staged once (STAGE_M) and shared, otherwise (tile_slot == -2) each
// particle reads its own matrix.  tile_slot == -1: no o-neighbour at all.
template <typename T, int TPN, bool STAGE_M>
__global__ __launch_bounds__(kBlock) void k_near(int n, int P, int nsp, const C2<T>* __restrict__ x,
                                                  C2<T>* __restrict__ y, const C2<T>* __restrict__ mats,
                                                  const int* __restrict__ nbr, const int* __restrict__ slot,
                                                  const int* __restrict__ tile_slot) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* xs = reinterpret_cast<C2<T>*>(smem_raw);  // [TPN][n]
  C2<T>* ms = xs + TPN * n;                         // [n][n]
  constexpr int PW = TPN / (kBlock / 64);
  const int tile = blockIdx.x, r = blockIdx.y;
  const int p0 = tile * TPN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j0 = lane, j1 = lane + 64;
  C2<T> a0[PW], a1[PW];
#pragma unroll
  for (int u = 0; u < PW; ++u) a0[u] = a1[u] = {0, 0};
  for (int o = 0; o < nsp; ++o) {
    const int ts = tile_slot[tile * nsp + o];
    if (ts == -1) continue;
    __syncthreads();
    for (int i = threadIdx.x; i < TPN * n; i += kBlock) {
      const int t = i / n, k = i - t * n;
      const int p = p0 + t;
      const int q = p < P ? nbr[p * nsp + o] : -1;
      xs[i] = q >= 0 ? x[((size_t)r * P + q) * n + k] : C2<T>{0, 0};
    }
    if (STAGE_M && ts >= 0)
      for (int i = threadIdx.x; i < n * n; i += kBlock) ms[i] = mats[(size_t)ts * n * n + i];
    __syncthreads();
    if (ts >= 0) {
      const C2<T>* __restrict__ M = STAGE_M ? ms : mats + (size_t)ts * n * n;
#pragma unroll 4
      for (int k = 0; k < n; ++k) {
        const C2<T> m0 = j0 < n ? M[k * n + j0] : C2<T>{0, 0};
        const C2<T> m1 = j1 < n ? M[k * n + j1] : C2<T>{0, 0};
#pragma unroll
        for (int u = 0; u < PW; ++u) {
          const C2<T> xv = xs[(wave * PW + u) * n + k];
          cfma(a0[u], m0, xv);
          cfma(a1[u], m1, xv);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < PW; ++u) {
        const int p = p0 + wave * PW + u;
        if (p >= P || nbr[p * nsp + o] < 0) continue;
        const C2<T>* __restrict__ M = mats + (size_t)slot[p * nsp + o] * n * n;
        for (int k = 0; k < n; ++k) {
          const C2<T> xv = xs[(wave * PW + u) * n + k];
          if (j0 < n) cfma(a0[u], M[k * n + j0], xv);
          if (j1 < n) cfma(a1[u], M[k * n + j1], xv);
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PW; ++u) {
    const int p = p0 + wave * PW + u;
    if (p >= P) continue;
    C2<T>* yp = y + ((size_t)r * P + p) * n;
    if (j0 < n) yp[j0] = a0[u];
    if (j1 < n) yp[j1] = a1[u];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill_zero(C2<T>* __restrict__ y, size_t count) {
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (; i < count; i += stride) y[i] = {0, 0};
}

// XCD-aware block order.  The dispatcher deals consecutive workgroups of a
// launch to the 8 XCDs in turn, and each XCD has its own L2.  A launch of
// 8 * ceil(total / 8) blocks renumbered this way gives XCD x the contiguous
// logical range [x * per, (x + 1) * per), so neighbouring tiles, which read
// the same inputs, share one L2.  Logical ids >= total are idle blocks.
__device__ __forceinline__ int xcd_block(int b, int total) {
  const int per = (total + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}
inline int xcd_grid(int total) { return 8 * ((total + 7) / 8); }

// ------------------------------------------------------------ MFMA GEMM --
// Real FP32 GEMM on the matrix cores, C[m][n] (+)= sum_k A[m][k] B[k][n],
// used for the dense contractions of the product (near blocks, leaf
// radiation, receive).  Complex matrices enter in real 2x2-block form: for
// a complex matrix Z the real matrix has Z_r, -Z_i in row 2i and Z_i, Z_r in
// row 2i+1, so that interleaved (re, im) vectors are its real operands.
//   A: row-major [M][lda].
//   B column n, segment s (K = nseg * kseg): floats Bsrc[bcol[n*nseg+s] *
//     ldb + k'] with k = s*kseg + k'; bcol < 0 gives a zero column.
//   C column n: floats Cdst[ccol[n] * ldc + m].
//   blockIdx.z = right-hand side r: B and C advance by strideB, strideC.
// Lane layout of v_mfma_f32_16x16x4f32: A[i][k] from lane i + 16k, B[k][j]
// from lane j + 16k, result row 4*(lane/16) + v, column lane % 16 in
// register v.
typedef float f32x4 __attribute__((ext_vector_type(4)));

// No LDS staging of the operands.  Block = 4 waves that
// share one output tile of RT x CT 16 x 16 MFMA tiles and split the K range
// four ways; partial sums are reduced through LDS in a fixed order.  K is
// walked in steps of 16 with a k-permutation inside each step: lane (i, kq)
// loads the 4 consecutive values k = 16 s + 4 kq + q (one 16-byte load) of
// its A row and B column, and MFMA q contracts over kq.  A and B use the same
// permutation, so the sum covers every k once.  Requires lda, ldb, kseg and
// the segment length multiples of 4 floats and 16-byte aligned bases.
//
// One launch runs up to two independent GEMMs (jobs): blocks [0, j0.tiles)
// take job 0, the rest job 1.  Within a job, block t computes row tile
// t % tiles_m of column tile t / tiles_m.  With a_off set, column tile nt
// multiplies A + a_off[nt] (one matrix per group of columns, e.g. per
// particle class, each group padded to whole column tiles).  Tag only gives
// each use its own kernel symbol.
struct GemmJob {
  const float* A;
  const int* a_off;
  const float* B;
  const int* bcol;  // B column n, segment s: floats B[bcol[n*nseg+s] * ldb + k'] (< 0: zero column)
  float* C;
  const int* ccol;  // C column n: floats C[ccol[n] * ldc + m] (< 0: not written)
  size_t sB, sC;    // per right-hand side strides of B and C
  int M, ncols, nseg, kseg, lda, ldb, ldc, acc, tiles_m, tiles;
  int fold;         // > 0: the right-hand sides are folded into the columns, column n = (n / fold, RHS
                    // n % fold), so that the tiles of one block share A over all RHS; 0: RHS = blockIdx.z
  int xcd;          // (job 0 only) blocks in XCD-aware order over the launch grid
  int wtile;        // 1: every wave of a block takes its own tile over all of K (short K); 0: the
                    // block's waves split one tile's K and add their partial sums
  const unsigned short* Ah;  // BF16-split kernel: A as BF16 heads and remainders (same layout as A)
  const unsigned short* Al;
};

constexpr int kMaxSeg = 9;  // segments of a gathered B column (the 3 x 3 neighbourhood)
constexpr int kGemmW = 8;   // waves per block of the FP32 GEMM launches
// blocks of a job: one per tile, or one per W tiles when every wave takes its own
__host__ __device__ inline int gemm_blocks(const GemmJob& j, int W) { return j.wtile ? (j.tiles + W - 1) / W : j.tiles; }
template <int RT, int CT, int Tag, int W>
__global__ __launch_bounds__(64 * W) void k_gemm_stream(GemmJob j0, GemmJob j1) {
  __shared__ f32x4 red[W - 1][RT * CT][64];
  __shared__ int sbc[16 * CT * kMaxSeg];  // the tile's source columns per segment (nseg > 1)
  const int nb0 = gemm_blocks(j0, W), nb1 = gemm_blocks(j1, W);
  const int bid = j0.xcd ? xcd_block(blockIdx.x, nb0 + nb1) : (int)blockIdx.x;
  if (bid >= nb0 + nb1) return;
  const bool second = bid >= nb0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wt = second ? j1.wtile : j0.wtile;
  const int t = wt ? (bid - (second ? nb0 : 0)) * W + wave : bid - (second ? nb0 : 0);
  if (wt && t >= (second ? j1.tiles : j0.tiles)) return;  // wave-tile blocks have no barrier
  const int M = second ? j1.M : j0.M, ncols = second ? j1.ncols : j0.ncols;
  const int nseg = second ? j1.nseg : j0.nseg, kseg = second ? j1.kseg : j0.kseg;
  const int lda = second ? j1.lda : j0.lda, ldb = second ? j1.ldb : j0.ldb, ldc = second ? j1.ldc : j0.ldc;
  const int accumulate = second ? j1.acc : j0.acc, tiles_m = second ? j1.tiles_m : j0.tiles_m;
  const int* __restrict__ bcol = second ? j1.bcol : j0.bcol;
  const int* __restrict__ ccol = second ? j1.ccol : j0.ccol;
  const int* __restrict__ a_off = second ? j1.a_off : j0.a_off;
  const int tm = t % tiles_m, tn = t / tiles_m;
  const int fold = second ? j1.fold : j0.fold, fd = fold > 0 ? fold : 1;
  const int m0 = tm * 16 * RT, n0 = tn * 16 * CT;
  // a_off has one entry per 16 (unfolded) columns; the CT tiles of a block
  // share it (the host keeps a block within one group)
  const float* __restrict__ A = (second ? j1.A : j0.A) + (a_off ? a_off[(n0 / fd) >> 4] : 0);
  const int i = lane & 15, kq = lane >> 4;
  const size_t sB = second ? j1.sB : j0.sB, sC = second ? j1.sC : j0.sC;
  const float* __restrict__ B0 = second ? j1.B : j0.B;
  const int K = nseg * kseg;
  const int nsup = (K + 15) / 16;
  const int s0 = wt ? 0 : (wave * nsup) / W, s1 = wt ? nsup : ((wave + 1) * nsup) / W;
  // this lane's columns: unfolded column and RHS, and their source columns
  // (one per column, or per segment staged in LDS: split-K blocks only, so
  // the barrier is uniform)
  int ncol[CT], src1[CT], rc[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int nf = n0 + 16 * ct + i;
    ncol[ct] = nf < ncols ? nf / fd : -1;
    rc[ct] = fold > 0 ? nf - (nf / fd) * fd : (int)blockIdx.z;
    src1[ct] = nseg == 1 && ncol[ct] >= 0 ? bcol[ncol[ct]] : -1;
  }
  if (nseg > 1) {
    for (int e = threadIdx.x; e < 16 * CT * nseg; e += 64 * W) {
      const int c = n0 + e / nseg;
      sbc[e] = c < ncols ? bcol[(size_t)(c / fd) * nseg + e % nseg] : -1;
    }
    __syncthreads();
  }
  f32x4 acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  // operands of k-step sup (16 k): A rows of this lane, B column of this lane
  auto load = [&](int sup, f32x4(&a)[RT], f32x4(&b)[CT]) {
    const int k = 16 * sup + 4 * kq;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int m = m0 + 16 * rt + i;
      a[rt] = (m < M && k < K) ? *reinterpret_cast<const f32x4*>(A + (size_t)m * lda + k) : f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      b[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (k < K) {
        const int sg = nseg == 1 ? 0 : k / kseg;
        const int src = nseg == 1 ? src1[ct] : sbc[(16 * ct + i) * nseg + sg];
        if (src >= 0)
          b[ct] = *reinterpret_cast<const f32x4*>(B0 + (size_t)rc[ct] * sB + (size_t)src * ldb + (k - sg * kseg));
      }
    }
  };
  // two-stage pipeline: the next step's loads are in flight during this
  // step's matrix-core products
  f32x4 a0[RT], b0[CT], a1[RT], b1[CT];
  if (s0 < s1) load(s0, a0, b0);
#pragma unroll 2
  for (int sup = s0; sup < s1; ++sup) {
    if (sup + 1 < s1) load(sup + 1, a1, b1);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[rt][q], b0[ct][q], acc[rt][ct], 0, 0, 0);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) a0[rt] = a1[rt];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) b0[ct] = b1[ct];
  }
  if (!wt) {
    if (wave > 0) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) red[wave - 1][rt * CT + ct][lane] = acc[rt][ct];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int w = 0; w < W - 1; ++w) acc[rt][ct] += red[w][rt * CT + ct][lane];
  }
  float* __restrict__ C0 = second ? j1.C : j0.C;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const f32x4 v = acc[rt][ct];
      const int n = ncol[ct];
      if (n < 0) continue;
      const int dcol = ccol[n];
      if (dcol < 0) continue;
      float* __restrict__ col = C0 + (size_t)rc[ct] * sC + (size_t)dcol * ldc;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + 16 * rt + 4 * kq + e;
        if (m < M) col[m] = accumulate ? col[m] + v[e] : v[e];
      }
    }
}

// y[r][p][:] = sum over the neighbours o of p of partial[r][o * P + p][:]
// (nf floats per particle, nf a multiple of 4), in a fixed order.  One lane
// per 4 floats; the nine partial loads are issued together (absent
// neighbours contribute exact zeros: their partial rows are never written).
__global__ __launch_bounds__(kBlock) void k_near_sum(int P, int nf, const float* __restrict__ partial,
                                                      const int* __restrict__ has, float* __restrict__ y) {
  const int nq = nf >> 2;
  const size_t cnt = (size_t)P * nq;
  const int r = blockIdx.y;
  const f32x4* __restrict__ pr = reinterpret_cast<const f32x4*>(partial) + (size_t)r * 9 * cnt;
  f32x4* __restrict__ yr = reinterpret_cast<f32x4*>(y) + (size_t)r * cnt;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < cnt; i += (size_t)gridDim.x * kBlock) {
    const int p = (int)(i / nq);
    f32x4 v[9];
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      v[o] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (has[p * 9 + o]) v[o] = pr[(size_t)o * cnt + i];
    }
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int o = 0; o < 9; ++o) acc += v[o];
    yr[i] = acc;
  }
}

// LDS-staged variant of k_gemm_stream for the FP32 jobs with the
// right-hand sides folded into the columns.  A block of W waves shares one
// A matrix (one column group): A passes through LDS in chunks of kLM rows
// by kLK k, and only the even rows of its real 2x2-block form are staged:
// row 2i holds (Re z, -Im z) of the complex entries z, and a lane rebuilds
// the real row it needs, (Re, -Im) for an even row or (Im, Re) for an odd
// one.  This halves the A bytes that leave L2.
//   MODE 0 (K <= kLK, one B segment): a wave keeps the B columns of its CT
//     column tiles in registers over all of K, reads them from memory once,
//     and walks the row chunks one 16-row tile at a time.
//   MODE 1 (M <= kLM): a wave keeps its C tiles (every row) in registers
//     and walks the k chunks; B is read once, its next chunk loaded
//     before the barrier that ends the current one.
// The next A chunk is loaded while the current one is multiplied; chunks
// alternate between two LDS buffers.  Every C tile is summed over k in
// increasing order by one wave, as in the one-wave tiles of k_gemm_stream.
// A block covers W * CT column tiles of 16 folded columns; the host keeps
// them inside one column group (W * CT divides the fold).  Requires M, K,
// kseg, lda, ldb and ldc multiples of 4 and 16-byte aligned bases.
constexpr int kLM = 128, kLK = 128, kLS4 = kLK / 4 + 1;  // f32x4 per staged row (one of padding)
__host__ __device__ inline int lds_mode(const GemmJob& j) {
  if (!j.A) return -1;
  if (j.nseg == 1 && j.kseg <= kLK) return 0;
  return j.M <= kLM ? 1 : -1;
}
// waves per block and column tiles per wave of the LDS kernel for R
// right-hand sides (W = 0: not applicable, k_gemm_stream runs the job)
inline void lds_config(int mode, int R, int& W, int& C) {
  W = C = 0;
  if (mode == 0 && R % 16 == 0) W = 8, C = 2;
  else if (R % 8 == 0) W = 8, C = 1;
  else if (R % 4 == 0) W = 4, C = 1;
}
__host__ __device__ inline int lds_blocks(const GemmJob& j, int W, int CT) {
  if (!j.A) return 0;
  const long long cols = (long long)j.ncols * (j.fold > 0 ? j.fold : 1);
  return (int)((cols + 16LL * W * CT - 1) / (16LL * W * CT));
}
__device__ __forceinline__ f32x4 expand_row(f32x4 v, bool odd) {
  // v = (Re z0, -Im z0, Re z1, -Im z1) from even row 2i; row 2i + 1 is
  // (Im z0, Re z0, Im z1, Re z1)
  return odd ? f32x4{-v[1], v[0], -v[3], v[2]} : v;
}
template <int MODE, int W, int CT, int Tag>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4))) void k_gemm_lds(GemmJob j0, GemmJob j1) {
  constexpr int NP = (kLM / 2) * (kLK / 4) / (64 * W);  // staged f32x4 per thread and chunk
  constexpr int NS = kLK / 16;                          // k-steps per chunk
  __shared__ f32x4 sA[2][kLM / 2][kLS4];
  // XCD-aware order per job: the hardware deals block b to XCD b % 8, and
  // each XCD takes an eighth of job 1's blocks, then an eighth of job 0's
  // (consecutive blocks of a job share their A matrix in that XCD's L2).
  // Splitting each job evenly keeps the XCDs balanced when the jobs' blocks
  // differ in cost (a projection block does eight times the work of a
  // near-block block).
  const int nb0 = lds_blocks(j0, W, CT), nb1 = lds_blocks(j1, W, CT);
  const int p0 = (nb0 + 7) >> 3, p1 = (nb1 + 7) >> 3;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const bool second = slot < p1;
  const int bl = second ? xcd * p1 + slot : xcd * p0 + (slot - p1);  // block within its job
  if (bl >= (second ? nb1 : nb0)) return;  // whole block
#define JF(f) (second ? j1.f : j0.f)
  const int M = JF(M), nseg = JF(nseg), kseg = JF(kseg), K = nseg * kseg;
  const int lda = JF(lda), ldb = JF(ldb), ldc = JF(ldc), accumulate = JF(acc), ncols = JF(ncols);
  const int fd = JF(fold) > 0 ? JF(fold) : 1;
  const int* __restrict__ bcol = JF(bcol);
  const int* __restrict__ ccol = JF(ccol);
  const int* __restrict__ a_off = JF(a_off);
  const size_t sB = JF(sB), sC = JF(sC);
  const float* __restrict__ B0 = JF(B);
  float* __restrict__ C0 = JF(C);
  const int nblk0 = bl * W * CT * 16;  // the block's first folded column
  const float* __restrict__ A = JF(A) + (a_off ? a_off[(nblk0 / fd) >> 4] : 0);
#undef JF
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
  const bool odd = i & 1;
  int base[CT], rc[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int n = nblk0 + (wave * CT + ct) * 16 + i, b = n / fd;
    base[ct] = b < ncols ? b : -1;
    rc[ct] = n - b * fd;
  }
  // A chunk: even rows m0 + 2 jr (jr < kLM / 2), k0 .. k0 + kLK
  f32x4 st[NP];
  auto stage_load = [&](int m0, int k0) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int p = threadIdx.x + u * 64 * W, jr = p / (kLK / 4), q = p % (kLK / 4);
      const int m = m0 + 2 * jr, k = k0 + 4 * q;
      // unconditional load from a clamped (valid) address, then a select:
      // no divergent branches around the staging registers
      const f32x4 v = *reinterpret_cast<const f32x4*>(A + (size_t)min(m, M - 2) * lda + min(k, K - 4));
      st[u] = (m < M && k < K) ? v : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto stage_store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int p = threadIdx.x + u * 64 * W;
      sA[buf][p / (kLK / 4)][p % (kLK / 4)] = st[u];
    }
  };
  // B of this lane's columns for the k-steps of chunk k0
  auto load_b = [&](int k0, f32x4(&b)[CT][NS]) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        // clamped indices and unconditional loads, as in the staging
        const int k = k0 + 16 * s + 4 * kq, kc = min(k, K - 4);
        const int sg = nseg == 1 ? 0 : kc / kseg;
        const int src = bcol[(size_t)max(base[ct], 0) * nseg + sg];
        const bool ok = base[ct] >= 0 && k < K && src >= 0;
        const f32x4 v = *reinterpret_cast<const f32x4*>(B0 + (size_t)rc[ct] * sB + (size_t)max(src, 0) * ldb +
                                                        (kc - sg * kseg));
        b[ct][s] = ok ? v : f32x4{0.f, 0.f, 0.f, 0.f};
      }
  };
  auto store_c = [&](int ct, int m, f32x4 v) {
    if (base[ct] < 0 || m >= M) return;
    const int dcol = ccol[base[ct]];
    if (dcol < 0) return;
    f32x4* dst = reinterpret_cast<f32x4*>(C0 + (size_t)rc[ct] * sC + (size_t)dcol * ldc + m);
    *dst = accumulate ? *dst + v : v;
  };
  f32x4 b[CT][NS];
  if constexpr (MODE == 0) {
    load_b(0, b);
    const int nmc = (M + kLM - 1) / kLM;
    stage_load(0, 0);
    stage_store(0);
    __syncthreads();
    for (int mc = 0; mc < nmc; ++mc) {
      const int buf = mc & 1;
      if (mc + 1 < nmc) stage_load((mc + 1) * kLM, 0);
      for (int rt = 0; rt < kLM / 16; ++rt) {
        const int mt = mc * kLM + 16 * rt;
        if (mt >= M) break;
        f32x4 acc[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (16 * s >= K) break;
          const f32x4 a = expand_row(sA[buf][8 * rt + (i >> 1)][4 * s + kq], odd);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
              acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], b[ct][s][q], acc[ct], 0, 0, 0);
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) store_c(ct, mt + 4 * kq, acc[ct]);
      }
      if (mc + 1 < nmc) {
        stage_store(buf ^ 1);
        __syncthreads();
      }
    }
  } else {
    constexpr int RT = kLM / 16;
    f32x4 acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nkc = (K + kLK - 1) / kLK;
    load_b(0, b);
    stage_load(0, 0);
    stage_store(0);
    __syncthreads();
    for (int kc = 0; kc < nkc; ++kc) {
      const int buf = kc & 1;
      if (kc + 1 < nkc) stage_load(0, (kc + 1) * kLK);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (kc * kLK + 16 * s >= K) break;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          if (16 * rt >= M) break;
          const f32x4 a = expand_row(sA[buf][8 * rt + (i >> 1)][4 * s + kq], odd);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
              acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], b[ct][s][q], acc[rt][ct], 0, 0, 0);
        }
        // one k-step's A reads at a time (hoisting all of a chunk's would
        // need more registers than four waves per SIMD have)
        __builtin_amdgcn_sched_barrier(0);
      }
      if (kc + 1 < nkc) {
        load_b((kc + 1) * kLK, b);  // in flight across the barrier
        stage_store(buf ^ 1);
        __syncthreads();
      }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) store_c(ct, 16 * rt + 4 * kq, acc[rt][ct]);
  }
}

// BF16-split variant: the same jobs, tiles and reduction as k_gemm_stream,
// with each FP32 product a b formed as a_h b_h + a_h b_l + a_l b_h from BF16
// heads and remainders (A split once on the host, B split in registers)
// on v_mfma_f32_16x16x16bf16_1k, accumulated in FP32.  Lane layout: A[i][k]
// is element k % 4 of lane i + 16 (k / 4), B[k][j] element k % 4 of lane
// j + 16 (k / 4); the result as for the FP32 instruction.  A lane loads the
// 4 consecutive k = 16 s + 4 kq .. + 3 of its row and column.
typedef short s16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {  // round to nearest, ties to even
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

template <int RT, int Tag>
__global__ __launch_bounds__(kBlock) void k_gemm_bf16x3(GemmJob j0, GemmJob j1) {
  __shared__ f32x4 red[3][RT][64];
  const int bid = j0.xcd ? xcd_block(blockIdx.x, j0.tiles + j1.tiles) : (int)blockIdx.x;
  if (bid >= j0.tiles + j1.tiles) return;
  const bool second = bid >= j0.tiles;
  const int t = second ? bid - j0.tiles : bid;
  const int M = second ? j1.M : j0.M, ncols = second ? j1.ncols : j0.ncols;
  const int nseg = second ? j1.nseg : j0.nseg, kseg = second ? j1.kseg : j0.kseg;
  const int lda = second ? j1.lda : j0.lda, ldb = second ? j1.ldb : j0.ldb, ldc = second ? j1.ldc : j0.ldc;
  const int accumulate = second ? j1.acc : j0.acc, tiles_m = second ? j1.tiles_m : j0.tiles_m;
  const int* __restrict__ bcol = second ? j1.bcol : j0.bcol;
  const int* __restrict__ ccol = second ? j1.ccol : j0.ccol;
  const int* __restrict__ a_off = second ? j1.a_off : j0.a_off;
  const int tm = t % tiles_m, tn = t / tiles_m;
  const size_t aoff = a_off ? (size_t)a_off[tn] : 0;
  const unsigned short* __restrict__ Ah = (second ? j1.Ah : j0.Ah) + aoff;
  const unsigned short* __restrict__ Al = (second ? j1.Al : j0.Al) + aoff;
  const int m0 = tm * 16 * RT, n0 = tn * 16, r = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  const float* __restrict__ Bb = (second ? j1.B : j0.B) + (size_t)r * (second ? j1.sB : j0.sB);
  const int K = nseg * kseg;
  const int nsup = (K + 15) / 16;
  const int s0 = (wave * nsup) / 4, s1 = ((wave + 1) * nsup) / 4;
  const int n = n0 + i;
  f32x4 acc[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int sup = s0; sup < s1; ++sup) {
    const int k = 16 * sup + 4 * kq;
    s16x4 ah[RT], al[RT], bh, bl;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int m = m0 + 16 * rt + i;
      const bool ok = m < M && k < K;
      ah[rt] = ok ? *reinterpret_cast<const s16x4*>(Ah + (size_t)m * lda + k) : s16x4{0, 0, 0, 0};
      al[rt] = ok ? *reinterpret_cast<const s16x4*>(Al + (size_t)m * lda + k) : s16x4{0, 0, 0, 0};
    }
    f32x4 b = f32x4{0.f, 0.f, 0.f, 0.f};
    if (n < ncols && k < K) {
      const int sg = nseg == 1 ? 0 : k / kseg;
      const int src = bcol[(size_t)n * nseg + sg];
      if (src >= 0) b = *reinterpret_cast<const f32x4*>(Bb + (size_t)src * ldb + (k - sg * kseg));
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const unsigned short h = f32_to_bf16(b[e]);
      bh[e] = (short)h;
      bl[e] = (short)f32_to_bf16(b[e] - bf16_to_f32(h));
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      acc[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[rt], bh, acc[rt], 0, 0, 0);
      acc[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[rt], bl, acc[rt], 0, 0, 0);
      acc[rt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[rt], bh, acc[rt], 0, 0, 0);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) red[wave - 1][rt][lane] = acc[rt];
  }
  __syncthreads();
  if (wave != 0 || n >= ncols) return;
  const int dcol = ccol[n];
  if (dcol < 0) return;
  float* __restrict__ col = (second ? j1.C : j0.C) + (size_t)r * (second ? j1.sC : j0.sC) + (size_t)dcol * ldc;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    f32x4 v = acc[rt];
#pragma unroll
    for (int w = 0; w < 3; ++w) v += red[w][rt][lane];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = m0 + 16 * rt + 4 * kq + e;
      if (m < M) col[m] = accumulate ? col[m] + v[e] : v[e];
    }
  }
}

// ------------------------------------------------------- leaf projection --
// U[r][box(p)][m] = sum_j Rm[class][j][m] x[r][p][j] for a tile of up to TP
// particles of one class; one thread per pattern sample m (blocks of 128
// samples along grid y).
constexpr int kProjBlock = 128;
template <typename T, int TP>
__global__ __launch_bounds__(kProjBlock) void k_project(int n, int P, int M2, int nbox, const C2<T>* __restrict__ x,
                                                         C2<T>* __restrict__ U, const C2<T>* __restrict__ Rm_all,
                                                         const int* __restrict__ rm_off, const int* __restrict__ order,
                                                         const int* __restrict__ tile_start,
                                                         const int* __restrict__ tile_count,
                                                         const int* __restrict__ tile_class,
                                                         const int* __restrict__ box_of) {
  extern __shared__ unsigned char smem_raw[];
  C2<T>* xs = reinterpret_cast<C2<T>*>(smem_raw);  // [TP][n]
  const int tile = blockIdx.x, r = blockIdx.z;
  const int cnt = tile_count[tile], st = tile_start[tile];
  const C2<T>* __restrict__ Rm = Rm_all + rm_off[tile_class[tile]];
  for (int i = threadIdx.x; i < TP * n; i += kProjBlock) {
    const int t = i / n, j = i - t * n;
    xs[i] = t < cnt ? x[((size_t)r * P + order[st + t]) * n + j] : C2<T>{0, 0};
  }
  __syncthreads();
  const int m = blockIdx.y * kProjBlock + threadIdx.x;
  if (m < M2) {
    C2<T> acc[TP];
#pragma unroll
    for (int t = 0; t < TP; ++t) acc[t] = {0, 0};
#pragma unroll 4
    for (int j = 0; j < n; ++j) {
      const C2<T> z = Rm[(size_t)j * M2 + m];
#pragma unroll
      for (int t = 0; t < TP; ++t) cfma(acc[t], z, xs[t * n + j]);
    }
#pragma unroll
    for (int t = 0; t < TP; ++t)
      if (t < cnt) U[((size_t)r * nbox + box_of[order[st + t]]) * M2 + m] = acc[t];
  }
}

// ---------------------------------------------------------------- receive --
// y[r][p][j] += sum_m Qm[class][m][j] G0[r][box(p)][m].  The tile's pattern
// samples are staged through LDS in chunks of MC; wave w handles particles
// w, w+4, ... of the tile; lane = output row (rows lane and lane + 64).
template <typename T, int TP>
__global__ __launch_bounds__(kBlock) void k_receive(int n, int P, int M2, int nbox, C2<T>* __restrict__ y,
                                                     const C2<T>* __restrict__ G, const C2<T>* __restrict__ Qm_all,
                                                     const int* __restrict__ qm_off, const int* __restrict__ order,
                                                     const int* __restrict__ tile_start, const int* __restrict__ tile_count,
                                                     const int* __restrict__ tile_class, const int* __restrict__ box_of) {
  constexpr int MC = 128;
  __shared__ C2<T> gs[TP * MC];
  const int tile = blockIdx.x, r = blockIdx.y;
  const int cnt = tile_count[tile], st = tile_start[tile];
  const C2<T>* __restrict__ Qm = Qm_all + qm_off[tile_class[tile]];
  constexpr int PW = TP / (kBlock / 64);  // particles per wave
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  C2<T> a0[PW], a1[PW];
#pragma unroll
  for (int u = 0; u < PW; ++u) a0[u] = a1[u] = {0, 0};
  const int j0 = lane, j1 = lane + 64;
  const bool two = n > 64;
  for (int m0 = 0; m0 < M2; m0 += MC) {
    const int mc = min(MC, M2 - m0);
    __syncthreads();
    for (int i = threadIdx.x; i < TP * MC; i += kBlock) {
      const int t = i / MC, m = i - t * MC;
      gs[i] = (t < cnt && m < mc) ? G[((size_t)r * nbox + box_of[order[st + t]]) * M2 + m0 + m] : C2<T>{0, 0};
    }
    __syncthreads();
    if (two) {
      for (int m = 0; m < mc; ++m) {
        const C2<T> q0 = j0 < n ? Qm[(size_t)(m0 + m) * n + j0] : C2<T>{0, 0};
        const C2<T> q1 = j1 < n ? Qm[(size_t)(m0 + m) * n + j1] : C2<T>{0, 0};
#pragma unroll
        for (int u = 0; u < PW; ++u) {
          const C2<T> g = gs[(wave + u * (kBlock / 64)) * MC + m];
          cfma(a0[u], q0, g);
          cfma(a1[u], q1, g);
        }
      }
    } else {
#pragma unroll 4
      for (int m = 0; m < mc; ++m) {
        const C2<T> q0 = j0 < n ? Qm[(size_t)(m0 + m) * n + j0] : C2<T>{0, 0};
#pragma unroll
        for (int u = 0; u < PW; ++u) cfma(a0[u], q0, gs[(wave + u * (kBlock / 64)) * MC + m]);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PW; ++u) {
    const int t = wave + u * (kBlock / 64);
    if (t >= cnt) continue;
    C2<T>* yp = y + ((size_t)r * P + order[st + t]) * n;
    if (j0 < n) { C2<T> v = yp[j0]; yp[j0] = {v.x + a0[u].x, v.y + a0[u].y}; }
    if (j1 < n) { C2<T> v = yp[j1]; yp[j1] = {v.x + a1[u].x, v.y + a1[u].y}; }
  }
}

// ------------------------------------------------- streamed interpolation --
// Aggregation and disaggregation as one pass over the rows of a pattern.
// A work item is one wave: (RHS, parent box, component, column strip, row
// chunk).  Its lanes hold SW columns of the output grid and, 32 lanes on,
// the SW columns half a turn further on in phi, so that a theta stencil
// crossing a pole, which reads its row at phi + pi, takes the partner
// lane's value (a lane exchange, no second read).  Where half a row has at
// most 16 columns (SW = 16) one wave takes both components.  The wave walks
// the extended rows of the input grid (the `order/2` pole reflections, the
// rows, the reflections at the other pole) once; per row it stages the phi
// windows of its columns of the four children (aggregation) or of the
// parent (disaggregation) in LDS, forms the phi stencil of each lane's
// column, and keeps the last `order` rows in registers, from which the theta
// stencil of every finished output row is formed.  Each input value is read
// once per item and each output written once; the next row's loads are in
// flight while a row is computed (two LDS buffers).
constexpr int kIStrip = 32;  // output columns per half-wave (16 when two components share a wave)
constexpr int kIStage = 8;   // staged values per lane and row, at most
template <typename T>
struct InterpArgs {
  const C2<T>* src;          // aggregation: child patterns; disaggregation: parent patterns
  C2<T>* dst;                // aggregation: parent patterns; disaggregation: child patterns (+=)
  const CP<T>* E;            // [K_p] exp(+jk khat . d) for the child offsets d = (+a/2, +a/2), (+a/2, -a/2)
  const int* chunk;          // aggregation: parent rows; disaggregation: extended child rows [nch + 1]
  const int* chunk_p;        // disaggregation: parent rows of each chunk [nch][2]
  const int* s0;             // [nt_p] first extended child row of each parent row's theta stencil
  const T* thw;              // [nt_p][order] theta weights (disaggregation: times wtheta_p / wtheta_c)
  const int* vrow;           // [nt_c + order] child row of each extended row
  const int* vflip;          // [nt_c + order] 1 where the extended row is a pole reflection
  const int* colb;           // [np_out] first input column of each output column's phi stencil
  const T* colw;             // [np_out][ntap] phi weights (disaggregation: times np_c / np_p)
  const int* wlo;            // [nst][2] first input column of each half-wave's window
  int nxc, nyc, ntc, npc, nxp, nyp, ntp, npp;
  int R, nst, nch, wlen, ntap;
};

template <typename T>
__device__ __forceinline__ C2<T> shfl_x32(C2<T> v) {
  return {__shfl_xor(v.x, 32), __shfl_xor(v.y, 32)};
}
// Read-only tables indexed uniformly over the wave (rows, stencil starts,
// theta weights), read through the constant address space so that they
// become scalar loads: a vector load of them would make the wave wait for
// every load in flight, the next row's prefetch included.
template <typename U>
__device__ __forceinline__ const __attribute__((address_space(4))) U* uni(const U* p) {
  return (const __attribute__((address_space(4))) U*)p;
}

// S_P = sum over the children q of phase_q . (Theta Phi S_q).  NE: the most
// parent rows whose theta stencil ends at one extended child row (2 on the
// excess-bandwidth grids, at most 3), the candidates whose phases each row
// loads ahead.
template <typename T, int ORD, int SW, int NE>
__global__ __launch_bounds__(64) void k_agg_stream(InterpArgs<T> A) {
  constexpr int G = kIStrip / SW;  // components per wave
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);  // [2 buffers][64 KS]: [G][4 children][2 halves][wlen]
  const int nbp = A.nxp * A.nyp, nbc = A.nxc * A.nyc;
  const int ncomp = 2 / G;
  const int total = A.R * nbp * ncomp * A.nst * A.nch;
  const int item = xcd_block(blockIdx.x, total);
  if (item >= total) return;
  int t = item;
  const int ch = t % A.nch;
  t /= A.nch;
  const int st = t % A.nst;
  t /= A.nst;
  const int comp0 = G == 2 ? 0 : t % 2;
  t /= ncomp;
  const int pb = t % nbp, r = t / nbp;
  const int lane = threadIdx.x, h = lane >> 5, g = (lane >> 4) & (G - 1), li = lane & (SW - 1);
  const int comp = comp0 + g;
  const int hp = A.npp >> 1, jj = st * SW + li;
  const bool valid = jj < hp;
  const int j = (valid ? jj : st * SW) + h * hp;  // idle lanes repeat the strip's first column
  const int Kc = A.ntc * A.npc, Kp = A.ntp * A.npp;
  const int wl = A.wlen, nbuf = G * 8 * wl;
  // this lane's phi stencil: ORD consecutive columns of its window
  T w[ORD];
#pragma unroll
  for (int b = 0; b < ORD; ++b) w[b] = A.colw[j * ORD + b];
  int off = A.colb[j] - uni(A.wlo)[st * 2 + h];
  if (off < 0) off += A.npc;
  const int lofs = ((g * 4) * 2 + h) * wl + off;  // + q * 2 * wl + buffer * nbuf
  // staging: value v of a row goes to buffer slot v = ((g * 4 + q) * 2 + hh) * wl + c;
  // its source as an offset into this RHS's child patterns.  With 32-column
  // strips the windows start at even columns and have even lengths, so a
  // lane stages two neighbouring columns with one 16-byte load (PR = 2
  // values per load; a pair never wraps round in phi, since the column
  // count is even)
  constexpr int KS = SW == kIStrip ? kIStage / 2 : 3 * kIStage / 4;
  constexpr int PR = SW == kIStrip ? 2 : 1, KL = KS / PR;  // values per load, loads per row
  using V = typename std::conditional<PR == 2, CP<T>, C2<T>>::type;
  const int PI = pb % A.nxp, PJ = pb / A.nxp;
  const C2<T>* __restrict__ srcr = A.src + (size_t)r * nbc * 2 * Kc;
  // (every lane loads and stores KL loads' values: a missing child or a slot
  // past the windows reads a valid address and stores zero, so that no load
  // is conditional and the next row's loads stay in flight)
  int so[KL];
  unsigned zmask = 0;
#pragma unroll
  for (int k = 0; k < KL; ++k) {
    const int v = PR * (lane + 64 * k);
    so[k] = 0;
    bool live = false;
    if (v < nbuf) {
      const int c = v % wl, rest = v / wl, hh = rest & 1, q = (rest >> 1) & 3, gg = rest >> 3;
      const int ci = 2 * PI + (q & 1), cj = 2 * PJ + (q >> 1);
      const int col = (uni(A.wlo)[st * 2 + hh] + c) % A.npc;
      if (ci < A.nxc && cj < A.nyc) {
        so[k] = (((cj * A.nxc + ci) * 2 + comp0 + gg) * Kc + col) / PR;  // even when PR = 2
        live = true;
      }
    }
    if (!live) zmask |= 1u << k;
  }
  const int p0 = uni(A.chunk)[ch], p1 = uni(A.chunk)[ch + 1];
  const int e0 = uni(A.s0)[p0], e1 = uni(A.s0)[p1 - 1] + ORD;
  const V* __restrict__ srcv = reinterpret_cast<const V*>(srcr);
  V nxt[KL];
  auto fetch = [&](int e) {
    const int ro = uni(A.vrow)[e] * A.npc / PR;
#pragma unroll
    for (int k = 0; k < KL; ++k) nxt[k] = at32(srcv, so[k] + ((zmask >> k) & 1 ? 0 : ro));
  };
  fetch(e0);
  C2<T> win[4][ORD];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int a = 0; a < ORD; ++a) win[q][a] = C2<T>{0, 0};
  C2<T>* __restrict__ outb = A.dst + ((size_t)r * nbp + pb) * 2 * Kp;  // this parent box's patterns
  const int oofs = comp * Kp + j;
  int pn = p0;
  // one extended row; row e0 + n * ORD + PH goes to window slot PH, so the
  // window (oldest row first) is slots PH + 1, ..., PH + ORD (mod ORD) and
  // rotates by renaming instead of moving registers (rows come ORD per
  // outer iteration, each at its compile-time phase)
  auto row = [&](auto phase, int e) {
    constexpr int PH = decltype(phase)::value;
    C2<T>* buf = lds + (e & 1) * 64 * KS;
    V* bufv = reinterpret_cast<V*>(buf);
#pragma unroll
    for (int k = 0; k < KL; ++k) bufv[lane + 64 * k] = (zmask >> k) & 1 ? V{} : nxt[k];
    // the phases of the parent rows this extended row finishes (loaded before
    // the next row's values, so that using them waits for these only)
    C2<T> ea1[NE], ea2[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int pu = min(pn + u, p1 - 1);
      const CP<T> e = at32(A.E, pu * A.npp + j);
      ea1[u] = e.a;
      ea2[u] = e.b;
    }
    if (e + 1 < e1) fetch(e + 1);
    __syncthreads();
    C2<T> f[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const C2<T>* __restrict__ lw = buf + lofs + q * 2 * wl;
      C2<T> v{0, 0};
#pragma unroll
      for (int b = 0; b < ORD; ++b) {
        const C2<T> z = lw[b];
        v.x = fmadd(w[b], z.x, v.x);
        v.y = fmadd(w[b], z.y, v.y);
      }
      f[q] = v;
    }
    if (uni(A.vflip)[e]) {
#pragma unroll
      for (int q = 0; q < 4; ++q) f[q] = shfl_x32(f[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) win[q][PH] = f[q];
    // parent rows whose theta stencil ends at this extended row (at most NE,
    // in order); the test is uniform over the wave, so only the rows that
    // end here are formed (their phases were loaded for all NE candidates,
    // unconditionally, ahead of the next row's values)
    int nemit = 0;
    pn = __builtin_amdgcn_readfirstlane(pn);  // uniform: the tests below branch on the scalar unit
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int pu = min(pn + u, p1 - 1);
      const bool ends = pn + u < p1 && uni(A.s0)[pn + u] + ORD - 1 == e;
      if (!ends) break;
      const auto tw = uni(A.thw) + pu * ORD;
      C2<T> v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v[q] = C2<T>{0, 0};
#pragma unroll
        for (int a = 0; a < ORD; ++a) {
          const C2<T> z = win[q][(PH + 1 + a) % ORD];
          v[q].x = fmadd(tw[a], z.x, v[q].x);
          v[q].y = fmadd(tw[a], z.y, v[q].y);
        }
      }
      // phases: child 3 = (+, +) -> E1, child 0 = conj(E1), child 1 =
      // (+, -) -> E2, child 2 = conj(E2)
      const C2<T> a1 = ea1[u], a2 = ea2[u];
      C2<T> o;
      o.x = a1.x * (v[3].x + v[0].x) - a1.y * (v[3].y - v[0].y) + a2.x * (v[1].x + v[2].x) - a2.y * (v[1].y - v[2].y);
      o.y = a1.x * (v[3].y + v[0].y) + a1.y * (v[3].x - v[0].x) + a2.x * (v[1].y + v[2].y) + a2.y * (v[1].x - v[2].x);
      if (valid) at32(outb, oofs + pu * A.npp) = o;
      ++nemit;
    }
    pn += nemit;
  };
  for (int e = e0; e < e1; e += ORD) {
    row(std::integral_constant<int, 0>{}, e);
    if (e + 1 < e1) row(std::integral_constant<int, 1>{}, e + 1);
    if (e + 2 < e1) row(std::integral_constant<int, 2>{}, e + 2);
    if (e + 3 < e1) row(std::integral_constant<int, 3>{}, e + 3);
    if constexpr (ORD > 4) {
      if (e + 4 < e1) row(std::integral_constant<int, 4 % ORD>{}, e + 4);
      if (e + 5 < e1) row(std::integral_constant<int, 5 % ORD>{}, e + 5);
    }
  }
}

// G_c += W_c^-1 I^T W_P (conj(phase_c) G_P) for the four children c of a
// parent box: the transposed stencils, streamed over the parent's rows.  A
// lane holds one child column (and its partner half a turn on); per parent
// row it forms the transposed phi stencil of the conjugate-phased parent row
// for each child, and adds it with the transposed theta weights into the
// `order` extended child rows that row reaches; an extended row is finished
// (added to the child's pattern) once no later parent row reaches it.  A
// pole reflection's sum belongs to the partner column's child row, which is
// the lane exchange of the transposed stencil.  Chunks own disjoint ranges
// of extended rows (the reflections with their rows).
template <typename T, int ORD, int NT, int SW>
__global__ __launch_bounds__(64) void k_dis_stream(InterpArgs<T> A) {
  constexpr int G = kIStrip / SW;
  extern __shared__ unsigned char smem_raw[];
  C2<T>* lds = reinterpret_cast<C2<T>*>(smem_raw);  // [2 buffers][G][4 children][2 halves][wlen]
  const int nbp = A.nxp * A.nyp, nbc = A.nxc * A.nyc;
  const int ncomp = 2 / G;
  const int total = A.R * nbp * ncomp * A.nst * A.nch;
  const int item = xcd_block(blockIdx.x, total);
  if (item >= total) return;
  int t = item;
  const int ch = t % A.nch;
  t /= A.nch;
  const int st = t % A.nst;
  t /= A.nst;
  const int comp0 = G == 2 ? 0 : t % 2;
  t /= ncomp;
  const int pb = t % nbp, r = t / nbp;
  const int lane = threadIdx.x, h = lane >> 5, g = (lane >> 4) & (G - 1), li = lane & (SW - 1);
  const int comp = comp0 + g;
  const int hc = A.npc >> 1, cc = st * SW + li;
  const bool valid = cc < hc;
  const int c = (valid ? cc : st * SW) + h * hc;  // idle lanes repeat the strip's first column
  const int Kc = A.ntc * A.npc, Kp = A.ntp * A.npp;
  const int wl = A.wlen, nbuf = G * 8 * wl;
  T w[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) w[k] = A.colw[c * NT + k];
  int off = A.colb[c] - uni(A.wlo)[st * 2 + h];
  if (off < 0) off += A.npp;
  const int lofs = (g * 4 * 2 + h) * wl + off;
  const int PI = pb % A.nxp, PJ = pb / A.nxp;
  // the four children's patterns at this lane's column, as offsets into
  // this RHS's child patterns (-1: no child, or an idle lane)
  C2<T>* __restrict__ dstr = A.dst + (size_t)r * nbc * 2 * Kc;
  int co[4];
  unsigned cmask = 0;  // children this lane writes
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ci = 2 * PI + (q & 1), cj = 2 * PJ + (q >> 1);
    const bool has = valid && ci < A.nxc && cj < A.nyc;
    co[q] = has ? ((cj * A.nxc + ci) * 2 + comp) * Kc + c : 0;
    if (has) cmask |= 1u << q;
  }
  // staging: parent value v of a row (component gg, half hh, window column
  // k) times the conjugate phases of the four children goes to slots
  // ((gg * 4 + q) * 2 + hh) * wl + k
  constexpr int KS = 3 * kIStage / 8;
  const int nv = G * 2 * wl;
  const C2<T>* __restrict__ gpr = A.src + ((size_t)r * nbp + pb) * 2 * Kp;
  // (every lane loads KS values; a value past the windows reads column 0
  // and goes to spare slots after the buffer, so that no load is
  // conditional and the next row's loads stay in flight)
  int scol[KS], sslot[KS], sgo[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int v = lane + 64 * k;
    scol[k] = 0;
    sslot[k] = nbuf + lane;
    sgo[k] = comp0 * Kp;
    if (v < nv) {
      const int kk = v % wl, rest = v / wl, hh = rest & 1, gg = rest >> 1;
      scol[k] = (uni(A.wlo)[st * 2 + hh] + kk) % A.npp;
      sslot[k] = (gg * 8 + hh) * wl + kk;
      sgo[k] = (comp0 + gg) * Kp + scol[k];
    }
  }
  const int E0 = uni(A.chunk)[ch], E1 = uni(A.chunk)[ch + 1];
  const int pfirst = uni(A.chunk_p)[2 * ch], plast = uni(A.chunk_p)[2 * ch + 1];
  const int half = ORD / 2, nvr = A.ntc + ORD;
  C2<T> ng[KS], ne1[KS], ne2[KS];
  auto fetch = [&](int p) {
    const int ro = p * A.npp;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      ng[k] = at32(gpr, sgo[k] + ro);
      const CP<T> e = at32(A.E, ro + scol[k]);
      ne1[k] = e.a;
      ne2[k] = e.b;
    }
  };
  fetch(pfirst);
  C2<T> acc[4][ORD];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int a = 0; a < ORD; ++a) acc[q][a] = C2<T>{0, 0};
  int ew = uni(A.s0)[pfirst];  // extended child row held in acc[.][0]
  // the oldest held row's translated child values: loaded once per parent
  // row, every row the same loads (so that the next row's loads, issued
  // after them, stay in flight while the flush waits for these)
  C2<T> pend[4];
  auto load_pend = [&]() {
    const int o = uni(A.vrow)[min(ew, nvr - 1)] * A.npc;
#pragma unroll
    for (int q = 0; q < 4; ++q) pend[q] = at32(dstr, co[q] + o);
  };
  load_pend();
  // adds the oldest held row to its child row (if this chunk owns it) and
  // shifts the window
  auto flush = [&]() {
    if (ew >= E0 && ew < E1) {
      const int o = uni(A.vrow)[ew] * A.npc;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if ((cmask >> q) & 1) at32(dstr, co[q] + o) = C2<T>{pend[q].x + acc[q][0].x, pend[q].y + acc[q][0].y};
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int a = 0; a + 1 < ORD; ++a) acc[q][a] = acc[q][a + 1];
      acc[q][ORD - 1] = C2<T>{0, 0};
    }
    ++ew;
  };
  for (int p = pfirst; p <= plast; ++p) {
    const int spp = uni(A.s0)[p];
    if (ew < spp) {
      flush();
      while (ew < spp) {  // a second row finished by the same parent row (rare)
        load_pend();
        flush();
      }
    }
    load_pend();
    C2<T>* buf = lds + (p & 1) * (nbuf + 6 * wl + 64);
    // child 0: E1 g, child 1: conj(E2) g, child 2: E2 g, child 3: conj(E1) g
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        C2<T>* d = buf + sslot[k];
        d[0] = cmul(ne1[k], ng[k]);
        d[2 * wl] = cmul_conj_a(ne2[k], ng[k]);
        d[4 * wl] = cmul(ne2[k], ng[k]);
        d[6 * wl] = cmul_conj_a(ne1[k], ng[k]);
      }
    fetch(min(p + 1, plast));
    __syncthreads();
    C2<T> f[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const C2<T>* __restrict__ lw = buf + lofs + q * 2 * wl;
      C2<T> v{0, 0};
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const C2<T> z = lw[k];
        v.x = fmadd(w[k], z.x, v.x);
        v.y = fmadd(w[k], z.y, v.y);
      }
      f[q] = v;
    }
    const auto tw = uni(A.thw) + p * ORD;
    if (spp < half || spp + ORD > half + A.ntc) {  // a tap on a pole reflection
      C2<T> gx[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) gx[q] = shfl_x32(f[q]);
#pragma unroll
      for (int a = 0; a < ORD; ++a) {
        const bool fl = uni(A.vflip)[spp + a] != 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const C2<T> z = fl ? gx[q] : f[q];
          acc[q][a].x = fmadd(tw[a], z.x, acc[q][a].x);
          acc[q][a].y = fmadd(tw[a], z.y, acc[q][a].y);
        }
      }
    } else {
#pragma unroll
      for (int a = 0; a < ORD; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[q][a].x = fmadd(tw[a], f[q].x, acc[q][a].x);
          acc[q][a].y = fmadd(tw[a], f[q].y, acc[q][a].y);
        }
    }
  }
  const int eend = min(E1, nvr);
  while (ew < eend) {
    flush();
    load_pend();
  }
}

// -------------------------------------------------------------- translate --
// G[r][p][c][s] = sum over the interaction list of TL[offset][s] S[r][q][c][s].
// The list of box p (at most 27 (source box, offset) pairs, built on the
// host) is uniform over the block, so all partner loads are independent.
// Blocks (box fastest, then RHS, then 256-sample chunk) in XCD-aware order.
constexpr int kMaxIL = 27;
// One translation level of a multi-level launch: its grid, sample count,
// patterns, operators and interaction lists, and its first block.
template <typename T>
struct TrLevel {
  const C2<T>* S;
  C2<T>* G;
  const C2<T>* TL;
  const int *il_cnt, *il_src, *il_off;
  int nx, ny, K, start;
  const CP<T>* TLp;  // FP32 register tiles: the 40 far offsets' operators in pairs, [20][K]
};
// The n-th of the 40 offsets (dx, dy) with |dx| or |dy| >= 2 in the 7 x 7
// block, in row order (dy outer, dx inner), as the index (dy + 3) * 7 + dx + 3
__host__ __device__ constexpr int tr_far_offset(int n) {
  for (int i = 0, m = 0; i < 49; ++i) {
    const int dx = i % 7 - 3, dy = i / 7 - 3;
    if (dx < -1 || dx > 1 || dy < -1 || dy > 1) {
      if (m == n) return i;
      ++m;
    }
  }
  return -1;
}
constexpr int kMaxTrLv = 12;
template <typename T>
struct TrLevels {
  TrLevel<T> lv[kMaxTrLv];
  int n, total;  // levels, blocks over all of them
};
// the level of block b (levels in order of their first block)
template <typename T>
__device__ __forceinline__ int tr_level(const TrLevels<T>& L, int b) {
  int l = 0;
  while (l + 1 < L.n && b >= L.lv[l + 1].start) ++l;
  return l;
}
// All levels in one launch: the translations of different levels are
// independent (each reads its own aggregated patterns).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_translate(TrLevels<T> L, int R) {
  const int gb = xcd_block(blockIdx.x, L.total);
  if (gb >= L.total) return;
  const TrLevel<T>& V = L.lv[tr_level(L, gb)];
  const int nb = V.nx * V.ny, K = V.K, lb = gb - V.start;
  const int p = lb % nb, rest = lb / nb;
  const int r = rest % R;
  const int s = (rest / R) * kBlock + threadIdx.x;
  if (s >= K) return;
  const int cnt = V.il_cnt[p];
  const C2<T>* __restrict__ Sr = V.S + (size_t)r * nb * 2 * K;
  const C2<T>* __restrict__ TL = V.TL;
  C2<T> g0{0, 0}, g1{0, 0};
#pragma unroll 4
  for (int e = 0; e < cnt; ++e) {
    const int q = V.il_src[p * kMaxIL + e], o = V.il_off[p * kMaxIL + e];
    const C2<T> t = TL[(size_t)o * K + s];
    const C2<T>* src = Sr + (size_t)q * 2 * K;
    cfma(g0, t, src[s]);
    cfma(g1, t, src[K + s]);
  }
  C2<T>* dst = V.G + ((size_t)r * nb + p) * 2 * K;
  dst[s] = g0;
  dst[K + s] = g1;
}

// The same sums with the partners staged in LDS.  The interaction list of a
// box is the 6 x 6 window of offsets [-2, 3] (even index) or [-3, 2] (odd)
// in x and y around it, without the 3 x 3 neighbourhood.  A block takes a
// TX x TY tile of receiving boxes, both components and NS consecutive
// samples: it stages the tile's (TX + 6) x (TY + 6) source boxes (zeros
// outside the grid) and the 49 translation operators of those samples, so
// each source sample is read from L2 once per tile instead of once per
// receiver.  Wave w takes the boxes of parity (w & 1, w >> 1), which makes
// its offset loop uniform.  The terms are added in the order of the
// gathered lists (dy outer, dx inner); partners outside the grid add zeros.
template <typename T>
struct TrNS {
  static constexpr int v = sizeof(T) == 4 ? 16 : 8;
};
// The sums of the boxes of parity (PX, PY) in the staged tile: all offsets
// are compile-time, so the stencil is 27 pairs of LDS reads at immediate
// offsets from one per-lane base.
template <typename T, int TX, int TY, int PX, int PY>
__device__ __forceinline__ void tr_tile_sums(const C2<T>* __restrict__ sS, const C2<T>* __restrict__ sT, int lane,
                                             int bx0, int by0, int s0, int nx, int ny, int K, C2<T>* __restrict__ Gr) {
  constexpr int NS = TrNS<T>::v, HX = TX + 6, BW = (TX / 2) * (TY / 2);
  constexpr int DXLO = PX ? -3 : -2, DYLO = PY ? -3 : -2;
  for (int it = lane; it < BW * NS; it += 64) {
    const int k = it / NS, s = it % NS;
    const int bx = 2 * (k % (TX / 2)) + PX, by = 2 * (k / (TX / 2)) + PY;
    const int gx = bx0 + bx, gy = by0 + by;
    if (gx >= nx || gy >= ny || s0 + s >= K) continue;
    const C2<T>* __restrict__ src = sS + 2 * ((by + 3) * HX + bx + 3) * NS + s;
    const C2<T>* __restrict__ tl = sT + s;
    C2<T> g0{0, 0}, g1{0, 0};
#pragma unroll
    for (int iy = 0; iy < 6; ++iy) {
#pragma unroll
      for (int ix = 0; ix < 6; ++ix) {
        const int dy = DYLO + iy, dx = DXLO + ix;
        if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
        const C2<T> t = tl[((dy + 3) * 7 + dx + 3) * NS];
        const int h = dy * HX + dx;
        cfma(g0, t, src[2 * h * NS]);
        cfma(g1, t, src[(2 * h + 1) * NS]);
      }
    }
    C2<T>* dst = Gr + (size_t)(gy * nx + gx) * 2 * K + s0 + s;
    dst[0] = g0;
    dst[K] = g1;
  }
}
// 16 bytes of complex values: the unit of the staging loads
template <typename T>
struct alignas(16) Vec16 {
  C2<T> c[16 / sizeof(C2<T>)];
};
// A block takes one tile and sample chunk for `rpb` consecutive RHS: the 49
// operators are staged once, and the next RHS's halo is loaded into
// registers while the current one is summed.
template <typename T, int TX, int TY>
__global__ __launch_bounds__(kBlock) void k_translate_tiled(TrLevels<T> L, int R, int rpb) {
  constexpr int NS = TrNS<T>::v, HX = TX + 6, HY = TY + 6;
  constexpr int VPU = 16 / sizeof(C2<T>), NV = NS / VPU;  // complex values per load, loads per row
  constexpr int NSL = HY * HX * 2 * NV, NTL = 49 * NV;    // loads of the halo and of the operators
  constexpr int IS = (NSL + kBlock - 1) / kBlock, IT = (NTL + kBlock - 1) / kBlock;
  static_assert(TX % 2 == 0 && TY % 2 == 0, "tiles start at even boxes");
  __shared__ Vec16<T> sSv[NSL];  // [halo box][component][sample]
  __shared__ Vec16<T> sTv[NTL];  // [offset][sample]
  const int gb = xcd_block(blockIdx.x, L.total);
  if (gb >= L.total) return;
  const TrLevel<T>& V = L.lv[tr_level(L, gb)];
  const int nx = V.nx, ny = V.ny, K = V.K, lb = gb - V.start;
  const C2<T>* __restrict__ S = V.S;
  C2<T>* __restrict__ G = V.G;
  const C2<T>* __restrict__ TL = V.TL;
  const int tx = (nx + TX - 1) / TX, ntile = tx * ((ny + TY - 1) / TY);
  const int nch = (K + NS - 1) / NS;
  const int tile = lb % ntile, rest = lb / ntile;
  const int ch = rest % nch, rg = rest / nch;
  const int r0 = rg * rpb, r1 = min(R, r0 + rpb);
  const int bx0 = (tile % tx) * TX, by0 = (tile / tx) * TY, s0 = ch * NS;
  const int nb = nx * ny;
  // this thread's halo loads: source offset within one RHS's patterns (-1:
  // outside the grid or past the pattern's end, a zero)
  int hoff[IS];
#pragma unroll
  for (int u = 0; u < IS; ++u) {
    const int i = threadIdx.x + u * kBlock;
    hoff[u] = -1;
    if (i < NSL) {
      const int s = (i % NV) * VPU, t = i / NV;
      const int h = t >> 1, gx = bx0 - 3 + h % HX, gy = by0 - 3 + h / HX;
      if (gx >= 0 && gy >= 0 && gx < nx && gy < ny && s0 + s < K)
        hoff[u] = ((gy * nx + gx) * 2 + (t & 1)) * K + s0 + s;
    }
  }
  Vec16<T> bs[IS];
  auto fetch = [&](int r) {
    const C2<T>* __restrict__ Sr = S + (size_t)r * nb * 2 * K;
#pragma unroll
    for (int u = 0; u < IS; ++u) bs[u] = hoff[u] >= 0 ? *reinterpret_cast<const Vec16<T>*>(Sr + hoff[u]) : Vec16<T>{};
  };
  fetch(r0);
  // the operators (K is even and chunks start at multiples of NS, so a
  // 16-byte unit never straddles the end of a pattern)
#pragma unroll
  for (int u = 0; u < IT; ++u) {
    const int i = threadIdx.x + u * kBlock;
    if (i < NTL) {
      const int s = (i % NV) * VPU, o = i / NV;
      sTv[i] = s0 + s < K ? *reinterpret_cast<const Vec16<T>*>(TL + (size_t)o * K + s0 + s) : Vec16<T>{};
    }
  }
  const C2<T>* __restrict__ sS = sSv[0].c;
  const C2<T>* __restrict__ sT = sTv[0].c;
  const int lane = threadIdx.x & 63;
  for (int r = r0; r < r1; ++r) {
    if (r > r0) __syncthreads();  // the previous RHS's sums have read the halo
#pragma unroll
    for (int u = 0; u < IS; ++u)
      if (threadIdx.x + u * kBlock < NSL) sSv[threadIdx.x + u * kBlock] = bs[u];
    if (r + 1 < r1) fetch(r + 1);
    __syncthreads();
    C2<T>* __restrict__ Gr = G + (size_t)r * nb * 2 * K;
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {  // wave index = box parity
      case 0: tr_tile_sums<T, TX, TY, 0, 0>(sS, sT, lane, bx0, by0, s0, nx, ny, K, Gr); break;
      case 1: tr_tile_sums<T, TX, TY, 1, 0>(sS, sT, lane, bx0, by0, s0, nx, ny, K, Gr); break;
      case 2: tr_tile_sums<T, TX, TY, 0, 1>(sS, sT, lane, bx0, by0, s0, nx, ny, K, Gr); break;
      default: tr_tile_sums<T, TX, TY, 1, 1>(sS, sT, lane, bx0, by0, s0, nx, ny, K, Gr); break;
    }
  }
}

// FP32 translation with no LDS: one wave per 4 x 4 tile of receiving boxes
// and 64 consecutive samples (one per lane).  A lane holds the 40 operators
// of its sample that a tile uses (offsets with |dx| or |dy| >= 2) and, one
// field component at a time, the 16 boxes' sums in registers, and reads
// each of the tile's 10 x 10 source boxes once per component; the interaction lists are known at compile time (a
// tile starts at even box indices, so a receiver's parity fixes its list).
// Terms are added in the order of the gathered lists (dy outer, dx inner).
constexpr int kTrRegTile = 4;
constexpr int kTrBand = 8;  // tile columns per band in the block order of k_translate_reg
__host__ __device__ constexpr bool tr_in_list(int rx, int ry, int dx, int dy) {
  return (dx < -1 || dx > 1 || dy < -1 || dy > 1) && dx >= ((rx & 1) ? -3 : -2) && dx <= ((rx & 1) ? 2 : 3) &&
         dy >= ((ry & 1) ? -3 : -2) && dy <= ((ry & 1) ? 2 : 3);
}
// One 4 x 4 tile of k_translate_reg, one field component at a time (16
// accumulators instead of 32 leave registers for source loads in flight).
// Sources are visited row by row, column by column, which keeps every
// receiver's terms in the order of its interaction list (dy outer, dx inner).
// The terms a source row adds to the tile's receivers:
// (CHECK: skip the source columns outside the grid; an interior tile has none)
template <bool CHECK>
__device__ __forceinline__ void tr_reg_row(C2<float> (&acc)[kTrRegTile * kTrRegTile], const C2<float> (&t)[7][7],
                                           const C2<float>* sv, int hy, int bx0, int nx) {
  constexpr int TT = kTrRegTile, H = TT + 6;
#pragma unroll
  for (int hx = 0; hx < H; ++hx) {
    const int gx = bx0 - 3 + hx;
    if (CHECK && (gx < 0 || gx >= nx)) continue;
#pragma unroll
    for (int ry = 0; ry < TT; ++ry)
#pragma unroll
      for (int rx = 0; rx < TT; ++rx) {
        const int dx = hx - 3 - rx, dy = hy - 3 - ry;
        if (dx < -3 || dx > 3 || dy < -3 || dy > 3 || !tr_in_list(rx, ry, dx, dy)) continue;
        cfma(acc[ry * TT + rx], t[dy + 3][dx + 3], sv[hx]);
      }
  }
}
// INTERIOR: the 10 x 10 source window lies inside the grid.  Its rows are
// loaded DEPTH rows ahead of the row being summed, with no bounds test
// between a load and its use (a load inside a conditional block makes the
// compiler wait for every outstanding load there).  CHK (a slower variant
// kept for measurement): a column test per source, a branch the compiler
// cannot remove, with a scheduling barrier after each row, holds the loads
// to that schedule; without it the compiler is free to issue all of a
// component's source loads at the top.
template <bool INTERIOR, int DEPTH, bool CHK>
__device__ __forceinline__ void tr_reg_tile(const C2<float>* Sr, C2<float>* __restrict__ Gr,
                                            const C2<float> (&t)[7][7], int bx0, int by0, int nx, int ny, int K,
                                            bool live) {
  constexpr int TT = kTrRegTile, H = TT + 6;
#pragma unroll 1
  for (int comp = 0; comp < 2; ++comp) {
    C2<float> acc[TT * TT];
#pragma unroll
    for (int b = 0; b < TT * TT; ++b) acc[b] = C2<float>{0.f, 0.f};
    const C2<float>* Sc = Sr + (size_t)comp * K;
    if constexpr (INTERIOR) {
      // rows DEPTH ahead of the one being summed, in a ring of DEPTH + 1
      C2<float> rb[DEPTH + 1][H];
      auto load_row = [&](int hy, C2<float>(&dst)[H]) {
        const C2<float>* row = Sc + ((size_t)(by0 - 3 + hy) * nx + (bx0 - 3)) * 2 * K;
#pragma unroll
        for (int hx = 0; hx < H; ++hx) dst[hx] = row[(size_t)hx * 2 * K];
      };
#pragma unroll
      for (int d = 0; d < DEPTH; ++d) load_row(d, rb[d]);
#pragma unroll
      for (int hy = 0; hy < H; ++hy) {
        if (hy + DEPTH < H) load_row(hy + DEPTH, rb[(hy + DEPTH) % (DEPTH + 1)]);
        tr_reg_row<CHK>(acc, t, rb[hy % (DEPTH + 1)], hy, bx0, nx);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int hy = 0; hy < H; ++hy) {
        const int gy = by0 - 3 + hy;
        if (gy < 0 || gy >= ny) continue;
        C2<float> sv[H];
        const C2<float>* row = Sc + ((size_t)gy * nx + (bx0 - 3)) * 2 * K;
#pragma unroll
        for (int hx = 0; hx < H; ++hx) {
          const int gx = bx0 - 3 + hx;
          sv[hx] = (gx >= 0 && gx < nx) ? row[(ptrdiff_t)hx * 2 * K] : C2<float>{0.f, 0.f};
        }
        tr_reg_row<true>(acc, t, sv, hy, bx0, nx);
      }
    }
    if (live) {
#pragma unroll
      for (int ry = 0; ry < TT; ++ry)
#pragma unroll
        for (int rx = 0; rx < TT; ++rx) {
          const int gx = bx0 + rx, gy = by0 + ry;
          if (!INTERIOR && (gx >= nx || gy >= ny)) continue;
          Gr[((size_t)gy * nx + gx) * 2 * K + (size_t)comp * K] = acc[ry * TT + rx];
        }
    }
  }
}
// operator pair Q of the far offsets into t (indices fixed at compile time,
// so that t stays in registers)
template <int Q>
__device__ __forceinline__ void tr_put_pair(C2<float> (&t)[7][7], CP<float> e) {
  constexpr int i0 = tr_far_offset(2 * Q), i1 = tr_far_offset(2 * Q + 1);
  t[i0 / 7][i0 % 7] = e.a;
  t[i1 / 7][i1 % 7] = e.b;
}
template <int... Q>
__device__ __forceinline__ void tr_load_ops(C2<float> (&t)[7][7], const CP<float>* p, int K,
                                            std::integer_sequence<int, Q...>) {
  const CP<float> e[] = {p[(size_t)Q * K]...};
  (tr_put_pair<Q>(t, e[Q]), ...);
}
template <int DEPTH, bool CHK>
__global__ __launch_bounds__(64) void k_translate_reg(TrLevels<float> L, int R) {
  constexpr int TT = kTrRegTile, H = TT + 6;
  const int gb = xcd_block(blockIdx.x, L.total);
  if (gb >= L.total) return;
  const TrLevel<float>& V = L.lv[tr_level(L, gb)];
  const int nx = V.nx, ny = V.ny, K = V.K, lb = gb - V.start;
  const int tx = (nx + TT - 1) / TT, ntile = tx * ((ny + TT - 1) / TT);
  // tile fastest, then sample chunk, then RHS (consecutive blocks of one tile
  // read neighbouring samples of the same boxes; ordering the RHS before the
  // chunks, so that one chunk of operators is read by the 16 RHS together,
  // measured 2% slower on the 200 x 200 lens)
  const int nch = (K + 63) / 64;
  const int tile = lb % ntile, rest = lb / ntile;
  const int ch = rest % nch, r = rest / nch;
  // tiles in vertical bands of kTrBand tile columns, row by row within a
  // band: a tile's upper neighbour (which shares 6 of its 10 source rows)
  // runs kTrBand blocks earlier instead of a whole tile row earlier, so the
  // shared rows are still in the XCD's L2
  const int ty = ntile / tx, nfull = tx / kTrBand;
  int tix, tiy;
  if (tile < nfull * kTrBand * ty) {
    const int band = tile / (kTrBand * ty), t2 = tile - band * kTrBand * ty;
    tix = band * kTrBand + t2 % kTrBand;
    tiy = t2 / kTrBand;
  } else {
    const int rem = tx - nfull * kTrBand, t3 = tile - nfull * kTrBand * ty;
    tix = nfull * kTrBand + t3 % rem;
    tiy = t3 / rem;
  }
  const int bx0 = tix * TT, by0 = tiy * TT;
  const int s = ch * 64 + (int)threadIdx.x;
  const bool live = s < K;
  const int sl = live ? s : K - 1;
  const size_t nb = (size_t)nx * ny;
  const C2<float>* Sr = V.S + (size_t)r * nb * 2 * K + sl;
  C2<float>* __restrict__ Gr = V.G + (size_t)r * nb * 2 * K + sl;
  // the 40 operators of this sample, two per 16-byte load
  C2<float> t[7][7];
#pragma unroll
  for (int dy = 0; dy < 7; ++dy)
#pragma unroll
    for (int dx = 0; dx < 7; ++dx) t[dy][dx] = C2<float>{0.f, 0.f};
  tr_load_ops(t, V.TLp + sl, K, std::make_integer_sequence<int, 20>{});
  // tiles whose 10 x 10 source window lies inside the grid take a path with
  // no bounds tests, so that no branch separates a load from its use and
  // the loads of later sources stay in flight (a load inside a conditional
  // block makes the compiler wait for every outstanding load there)
  if (bx0 >= 3 && by0 >= 3 && bx0 + TT + 3 <= nx && by0 + TT + 3 <= ny)
    tr_reg_tile<true, DEPTH, CHK>(Sr, Gr, t, bx0, by0, nx, ny, K, live);
  else
    tr_reg_tile<false, DEPTH, CHK>(Sr, Gr, t, bx0, by0, nx, ny, K, live);
}

// ----------------------------------------------------------------- fields --
// Scattered E at observation points from the leaf patterns U_p (the
// projection of x): the far interaction of the product with the observation
// point as a receiving box of zero size,
//   E(r) = -jk sum_p sum_s w_s T_L(khat_s, r - c_p) (U_th,p(s) th_s + U_ph,p(s) ph_s),
// valid where r is farther from c_p than the particle's circumscribed
// radius.  Block = kFldPts points x one RHS; thread = one sample s of the
// leaf sphere (K <= kBlock).  Per chunk of kFldPar particles the block
// stages, for every (point, particle) pair, the unit vector and the Hankel
// coefficients -jk/(16 pi^2) (-j)^l (2l+1) h_l^(2)(k|D|) (FP64 recurrence,
// stored FP32); each thread then sums its sample's Legendre series.
constexpr int kFldPts = 8, kFldPar = 32, kFldMaxL = 16;
static_assert(kFldPts * kFldPar == kBlock, "one (point, particle) pair per thread in the staging");
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fields(int P, int K, int L, double k, const double* __restrict__ centers,
                                                    const int* __restrict__ box_of, int nb0,
                                                    const C2<T>* __restrict__ S0, const float* __restrict__ tab,
                                                    int npts, const double* __restrict__ pts, C2<T>* __restrict__ E) {
  __shared__ float2 cl[kFldPts * kFldPar][kFldMaxL + 1];
  __shared__ float dh[kFldPts * kFldPar][3];
  __shared__ float2 red[kBlock / 64][kFldPts * 3];
  const int r = blockIdx.y, pt0 = blockIdx.x * kFldPts;
  const int s = threadIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool live = s < K;
  float ks[3] = {0, 0, 0};
  if (live)
    for (int c = 0; c < 3; ++c) ks[c] = tab[s * 10 + c];
  C2<float> acc[kFldPts][2];  // per point: sums of T U_th and T U_ph
#pragma unroll
  for (int q = 0; q < kFldPts; ++q) acc[q][0] = acc[q][1] = C2<float>{0.f, 0.f};
  const C2<T>* __restrict__ Sr = S0 + (size_t)r * nb0 * 2 * K;
  for (int pc = 0; pc < P; pc += kFldPar) {
    __syncthreads();  // the previous chunk's coefficients are consumed
    {
      const int q = threadIdx.x / kFldPar, j = threadIdx.x % kFldPar;  // kBlock = kFldPts * kFldPar
      const int p = pc + j, pt = pt0 + q;
      if (p < P && pt < npts) {
        const double dx = pts[3 * pt] - centers[3 * p], dy = pts[3 * pt + 1] - centers[3 * p + 1],
                     dz = pts[3 * pt + 2] - centers[3 * p + 2];
        const double D = sqrt(dx * dx + dy * dy + dz * dz), x = k * D;
        dh[threadIdx.x][0] = (float)(dx / D);
        dh[threadIdx.x][1] = (float)(dy / D);
        dh[threadIdx.x][2] = (float)(dz / D);
        // h_0 = j e^{-jx}/x, h_1 = e^{-jx}(j/x^2 - 1/x), h_{l+1} = (2l+1)/x h_l - h_{l-1}
        const double cx = cos(x), sx = sin(x);  // e^{-jx} = cx - j sx
        double h0r = sx / x, h0i = cx / x;
        double h1r = sx / (x * x) - cx / x, h1i = cx / (x * x) + sx / x;
        const double pr = 0.0, pi = -k / (16.0 * 3.14159265358979323846 * 3.14159265358979323846);  // -jk/(16 pi^2)
        for (int l = 0; l <= L; ++l) {
          double hr, hi;
          if (l == 0) {
            hr = h0r;
            hi = h0i;
          } else if (l == 1) {
            hr = h1r;
            hi = h1i;
          } else {
            hr = (2.0 * l - 1.0) / x * h1r - h0r;
            hi = (2.0 * l - 1.0) / x * h1i - h0i;
            h0r = h1r;
            h0i = h1i;
            h1r = hr;
            h1i = hi;
          }
          // (-j)^l (2l+1) h_l, times the prefactor
          double ar = (2.0 * l + 1.0) * hr, ai = (2.0 * l + 1.0) * hi, t;
          switch (l & 3) {
            case 1: t = ar; ar = ai; ai = -t; break;   // times -j
            case 2: ar = -ar; ai = -ai; break;
            case 3: t = ar; ar = -ai; ai = t; break;   // times +j
            default: break;
          }
          cl[threadIdx.x][l] = make_float2((float)(pr * ar - pi * ai), (float)(pr * ai + pi * ar));
        }
      } else {
        dh[threadIdx.x][0] = dh[threadIdx.x][1] = dh[threadIdx.x][2] = 0.f;
        for (int l = 0; l <= L; ++l) cl[threadIdx.x][l] = make_float2(0.f, 0.f);
      }
    }
    __syncthreads();
    if (!live) continue;
    const int nj = min(kFldPar, P - pc);
    for (int j = 0; j < nj; ++j) {
      const int p = pc + j;
      const C2<T>* Up = Sr + (size_t)box_of[p] * 2 * K;
      const C2<float> ut{(float)Up[s].x, (float)Up[s].y}, up{(float)Up[K + s].x, (float)Up[K + s].y};
#pragma unroll
      for (int q = 0; q < kFldPts; ++q) {
        const int e = q * kFldPar + j;
        const float mu = ks[0] * dh[e][0] + ks[1] * dh[e][1] + ks[2] * dh[e][2];
        // T = sum_l c_l P_l(mu) by the Legendre recurrence
        float p0 = 1.f, p1 = mu;
        float2 c = cl[e][0];
        C2<float> tt{c.x, c.y};
        c = cl[e][1];
        tt.x = fmadd(c.x, p1, tt.x);
        tt.y = fmadd(c.y, p1, tt.y);
        for (int l = 1; l < L; ++l) {
          const float p2 = ((2.f * l + 1.f) * mu * p1 - (float)l * p0) / (float)(l + 1);
          c = cl[e][l + 1];
          tt.x = fmadd(c.x, p2, tt.x);
          tt.y = fmadd(c.y, p2, tt.y);
          p0 = p1;
          p1 = p2;
        }
        cfma(acc[q][0], tt, ut);
        cfma(acc[q][1], tt, up);
      }
    }
  }
  // E += -jk w_s (A th_s + B ph_s), summed over the samples (threads)
  float th[3] = {0, 0, 0}, ph[3] = {0, 0, 0}, ws = 0;
  if (live) {
    for (int c = 0; c < 3; ++c) {
      th[c] = tab[s * 10 + 3 + c];
      ph[c] = tab[s * 10 + 6 + c];
    }
    ws = tab[s * 10 + 9];
  }
  const float kf = (float)k;
#pragma unroll
  for (int q = 0; q < kFldPts; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // v = A th_c + B ph_c, times -jk w_s
      const float vx = acc[q][0].x * th[c] + acc[q][1].x * ph[c], vy = acc[q][0].y * th[c] + acc[q][1].y * ph[c];
      float ox = kf * ws * vy, oy = -kf * ws * vx;
      for (int o = 32; o > 0; o >>= 1) {
        ox += __shfl_xor(ox, o);
        oy += __shfl_xor(oy, o);
      }
      if (lane == 0) red[wave][q * 3 + c] = make_float2(ox, oy);
    }
  __syncthreads();
  if (threadIdx.x < kFldPts * 3) {
    const int q = threadIdx.x / 3, c = threadIdx.x % 3, pt = pt0 + q;
    if (pt < npts) {
      float2 o = make_float2(0.f, 0.f);
      for (int w = 0; w < kBlock / 64; ++w) {
        o.x += red[w][threadIdx.x].x;
        o.y += red[w][threadIdx.x].y;
      }
      E[((size_t)r * npts + pt) * 3 + c] = C2<T>{(T)o.x, (T)o.y};
    }
  }
}

// -------------------------------------------------------------------- rhs --
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rhs(int n, int P, int R, const C2<T>* __restrict__ pat,
                                                 const int* __restrict__ class_of, const C2<T>* __restrict__ phase,
                                                 C2<T>* __restrict__ b) {
  const size_t total = (size_t)R * P * n;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (size_t)gridDim.x * kBlock) {
    const int j = (int)(i % n);
    const size_t rp = i / n;
    const int p = (int)(rp % P), r = (int)(rp / P);
    const C2<T> v = cmul(phase[rp], pat[((size_t)class_of[p] * R + r) * n + j]);
    b[i] = {-v.x, -v.y};
  }
}

// ------------------------------------------------ FP64 GMRES vector kernels --
using Z = C2<double>;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_z(const C2<T>* __restrict__ a, Z* __restrict__ b, size_t cnt) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < cnt; i += (size_t)gridDim.x * kBlock)
    b[i] = {(double)a[i].x, (double)a[i].y};
}
template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_convert(const C2<S>* __restrict__ a, C2<D>* __restrict__ b, size_t cnt) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < cnt; i += (size_t)gridDim.x * kBlock)
    b[i] = {(D)a[i].x, (D)a[i].y};
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_from_z(const Z* __restrict__ a, C2<T>* __restrict__ b, size_t cnt) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < cnt; i += (size_t)gridDim.x * kBlock)
    b[i] = {(T)a[i].x, (T)a[i].y};
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

constexpr int kDotE = 4;  // vector elements per lane and sweep of k_dots
constexpr int kDotMaxBlocks = 512;
constexpr int kDotMinBlocks = 2048;  // blocks k_dots aims for, over stretches and vector groups

// Block partial sums of the inner products conj(V_i) . w (slots i < nv) and,
// when want_norm, of |w|^2 (slot nv), in one sweep over the basis (stored
// in VB precision, products accumulated in FP64).  Grid: stretches of w x
// groups of gsz basis vectors x RHS (the norm goes with group 0), so that a
// short basis still fills the chip.  The four waves of a block share one
// stretch of w; partial[((r * ldp) + slot) * gridDim.x + blockIdx.x].  RHS r
// is skipped where gate[r] == 0.  With jd, the basis has *jd + 1 vectors
// (the Arnoldi step index on the device) and the group size is derived
// from it as the host derives it (dot_group); groups past the basis exit.
template <typename VB>
constexpr int dot_vu() { return 4; }  // basis vectors loaded per step
// vectors per group for nv basis vectors: at most gcap groups (the number
// of w stretches that makes kDotMinBlocks blocks), each a multiple of VU
__host__ __device__ inline int dot_group(int nv, int VU, int gcap) {
  const int steps = (nv + VU - 1) / VU;
  const int want = steps < gcap ? (steps > 1 ? steps : 1) : (gcap > 1 ? gcap : 1);
  return VU * ((steps + want - 1) / want);
}
template <typename VB>
__global__ __launch_bounds__(kBlock) void k_dots(int nv, int want_norm, int gsz, int gcap, size_t Nt, size_t vstride,
                                                  const C2<VB>* __restrict__ V, const Z* __restrict__ w,
                                                  Z* __restrict__ partial, int ldp, const int* __restrict__ gate,
                                                  const int* __restrict__ jd) {
  const int r = blockIdx.z;
  if (gate && !gate[r]) return;
  if (jd) {
    nv = *jd + 1;
    gsz = dot_group(nv, dot_vu<VB>(), gcap);
  }
  // per wave: its stretches of w (E elements per lane and sweep) against
  // the group's basis vectors; the wave's sum for each vector goes to LDS
  // red[vector][wave] (dynamic, (gsz + want_norm) * kBlock / 64 entries)
  extern __shared__ unsigned char smem_raw[];
  Z* red = reinterpret_cast<Z*>(smem_raw);
  constexpr int NW = kBlock / 64;
  constexpr int VU = dot_vu<VB>(), E = kDotE;  // basis vectors per step, elements per lane
  const int v0 = blockIdx.y * gsz;
  const int cnt = min(gsz, nv - v0), norm = want_norm && blockIdx.y == 0;
  if (cnt <= 0 && !norm) return;
  const int ns = cnt + norm, nblk = gridDim.x, blk = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < ns * NW; i += kBlock) red[i] = Z{0, 0};
  __syncthreads();
  const Z* wr = w + (size_t)r * Nt;
  const C2<VB>* Vr = V + (size_t)r * Nt + (size_t)v0 * vstride;
  const size_t sweep = (size_t)nblk * NW * 64 * E;
  const size_t first = ((size_t)blk * NW + wave) * 64 * E;
  // per step of VU basis vectors, each lane sums its elements over all of
  // the wave's sweeps first and the wave reduces once per vector (a wave
  // reduction costs a chain of six cross-lane exchanges; one per sweep made
  // the pass four times slower than the subtraction pass over the same
  // basis); the wave's stretch of w is re-read per step from L2
  for (int i0 = 0; i0 < cnt; i0 += VU) {
    double ax[VU], ay[VU];
#pragma unroll
    for (int u = 0; u < VU; ++u) ax[u] = ay[u] = 0;
    for (size_t base = first; base < Nt; base += sweep) {
      Z wv[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const size_t k = base + (size_t)e * 64 + lane;
        wv[e] = k < Nt ? wr[k] : Z{0, 0};
      }
      C2<VB> v[VU][E];
#pragma unroll
      for (int u = 0; u < VU; ++u)
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const size_t k = base + (size_t)e * 64 + lane;
          v[u][e] = (i0 + u < cnt && k < Nt) ? Vr[(size_t)(i0 + u) * vstride + k] : C2<VB>{0, 0};
        }
#pragma unroll
      for (int u = 0; u < VU; ++u)
#pragma unroll
        for (int e = 0; e < E; ++e) {  // conj(v) w
          const double a = (double)v[u][e].x, b = (double)v[u][e].y;
          ax[u] += a * wv[e].x + b * wv[e].y;
          ay[u] += a * wv[e].y - b * wv[e].x;
        }
    }
#pragma unroll
    for (int u = 0; u < VU; ++u) {
      const double sx = wave_sum(ax[u]), sy = wave_sum(ay[u]);
      if (lane == 0 && i0 + u < cnt) red[(i0 + u) * NW + wave] = Z{sx, sy};
    }
  }
  if (norm) {
    double nn = 0;
    for (size_t base = first; base < Nt; base += sweep) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const size_t k = base + (size_t)e * 64 + lane;
        const Z z = k < Nt ? wr[k] : Z{0, 0};
        nn += z.x * z.x + z.y * z.y;
      }
    }
    nn = wave_sum(nn);
    if (lane == 0) red[cnt * NW + wave] = Z{nn, 0};
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ns; i += kBlock) {
    Z o{0, 0};
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      o.x += red[i * NW + q].x;
      o.y += red[i * NW + q].y;
    }
    partial[((size_t)r * ldp + (i < cnt ? v0 + i : nv)) * nblk + blk] = o;
  }
}

// out[r * ldo + s] = sum over b < nblk of partial[((r * ldp) + s) * nblk + b]
// (grid: slots x R), in a fixed order.
// Per-RHS block partials of y^H b (slot 0) and |y|^2 (slot 1), reduced by
// k_reduce: the minimal-residual scaling of an initial guess.
__global__ __launch_bounds__(kBlock) void k_guess_dots(size_t Nt, const Z* __restrict__ y, const Z* __restrict__ b,
                                                        Z* __restrict__ partial) {
  const int r = blockIdx.y, nblk = gridDim.x, blk = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __shared__ double red[3][kBlock / 64];
  const Z* yr = y + (size_t)r * Nt;
  const Z* br = b + (size_t)r * Nt;
  double px = 0, py = 0, nn = 0;
  for (size_t k = (size_t)blk * kBlock + threadIdx.x; k < Nt; k += (size_t)nblk * kBlock) {
    const Z a = yr[k], c = br[k];
    px += a.x * c.x + a.y * c.y;
    py += a.x * c.y - a.y * c.x;
    nn += a.x * a.x + a.y * a.y;
  }
  px = wave_sum(px);
  py = wave_sum(py);
  nn = wave_sum(nn);
  if (lane == 0) {
    red[0][wave] = px;
    red[1][wave] = py;
    red[2][wave] = nn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sx = 0, sy = 0, sn = 0;
    for (int q = 0; q < kBlock / 64; ++q) {
      sx += red[0][q];
      sy += red[1][q];
      sn += red[2][q];
    }
    partial[((size_t)r * 2 + 0) * nblk + blk] = Z{sx, sy};
    partial[((size_t)r * 2 + 1) * nblk + blk] = Z{sn, 0.0};
  }
}
// x_r = a_r x_r and w_r = b_r - a_r y_r (y = A x before scaling)
__global__ __launch_bounds__(kBlock) void k_guess_apply(size_t Nt, const Z* __restrict__ alpha, Z* __restrict__ x,
                                                         const Z* __restrict__ y, const Z* __restrict__ b,
                                                         Z* __restrict__ w) {
  const int r = blockIdx.y;
  const Z a = alpha[r];
  for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < Nt; k += (size_t)gridDim.x * kBlock) {
    const size_t i = (size_t)r * Nt + k;
    const Z xv = x[i], yv = y[i], bv = b[i];
    x[i] = Z{a.x * xv.x - a.y * xv.y, a.x * xv.y + a.y * xv.x};
    w[i] = Z{bv.x - (a.x * yv.x - a.y * yv.y), bv.y - (a.x * yv.y + a.y * yv.x)};
  }
}
__global__ __launch_bounds__(kBlock) void k_reduce(int nblk, const Z* __restrict__ partial, int ldp,
                                                    Z* __restrict__ out, int ldo, const int* __restrict__ gate,
                                                    const int* __restrict__ jd, int extra) {
  const int s = blockIdx.x, r = blockIdx.y;
  if (gate && !gate[r]) return;
  if (jd && s >= *jd + 1 + extra) return;  // slots: *jd + 1 dots, then `extra` more
  __shared__ double red[2][kBlock / 64];
  const Z* p = partial + ((size_t)r * ldp + s) * nblk;
  double ax = 0, ay = 0;
  for (int b = threadIdx.x; b < nblk; b += kBlock) {
    ax += p[b].x;
    ay += p[b].y;
  }
  ax = wave_sum(ax);
  ay = wave_sum(ay);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    red[0][wave] = ax;
    red[1][wave] = ay;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Z o{0, 0};
    for (int q = 0; q < kBlock / 64; ++q) {
      o.x += red[0][q];
      o.y += red[1][q];
    }
    out[(size_t)r * ldo + s] = o;
  }
}

// w[r] -= sum_{i<nv} V_i[r] c[r][i]; block partial sums of |w[r]|^2 after the
// update go to partial[r * gridDim.x + blockIdx.x] (imaginary part 0).
template <typename VB>
__global__ __launch_bounds__(kBlock) void k_subtract_norm(int nv, size_t Nt, size_t vstride, const C2<VB>* __restrict__ V,
                                                           const Z* __restrict__ c, int ldc, Z* __restrict__ w,
                                                           Z* __restrict__ partial, const int* __restrict__ gate,
                                                           const int* __restrict__ jd) {
  const int r = blockIdx.y;
  if (gate && !gate[r]) return;
  if (jd) nv = *jd + 1;
  __shared__ double red[kBlock / 64];
  constexpr int VU = sizeof(VB) == 4 ? 8 : 4;  // basis vectors loaded together
  const Z* cr = c + (size_t)r * ldc;
  Z* wr = w + (size_t)r * Nt;
  const C2<VB>* Vr = V + (size_t)r * Nt;
  double s2 = 0;
  for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < Nt; k += (size_t)gridDim.x * kBlock) {
    Z acc = wr[k];
    int i = 0;
    for (; i + VU <= nv; i += VU) {
      Z v[VU];
#pragma unroll
      for (int u = 0; u < VU; ++u) {
        const C2<VB> t = Vr[(size_t)(i + u) * vstride + k];
        v[u] = Z{(double)t.x, (double)t.y};
      }
#pragma unroll
      for (int u = 0; u < VU; ++u) {
        const Z q = cr[i + u];
        acc.x -= v[u].x * q.x - v[u].y * q.y;
        acc.y -= v[u].x * q.y + v[u].y * q.x;
      }
    }
    for (; i < nv; ++i) {
      const C2<VB> t = Vr[(size_t)i * vstride + k];
      const Z v{(double)t.x, (double)t.y}, q = cr[i];
      acc.x -= v.x * q.x - v.y * q.y;
      acc.y -= v.x * q.y + v.y * q.x;
    }
    wr[k] = acc;
    s2 += acc.x * acc.x + acc.y * acc.y;
  }
  s2 = wave_sum(s2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = 0;
    for (int q = 0; q < kBlock / 64; ++q) o += red[q];
    partial[(size_t)r * gridDim.x + blockIdx.x] = Z{o, 0};
  }
}

// Selective reorthogonalisation (Daniel-Gragg-Kaufman-Stewart): a second
// Gram-Schmidt pass is taken where the first removed more than half of
// |w|^2, i.e. |w'| < |w| / sqrt(2); always when `always`.
__global__ void k_dgks_gate(int R, const Z* __restrict__ h1, int ld, int nv, const Z* __restrict__ n1,
                            int* __restrict__ gate, int always, const int* __restrict__ jd) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  if (jd) nv = *jd + 1;
  gate[r] = (always || n1[r].x < 0.5 * h1[(size_t)r * ld + nv].x) ? 1 : 0;
}

// Hessenberg column: col[r][i] = h1 + h2 (i < nv), col[r][nv] = |w| after the
// last pass, col[r][nv+1] = gate; scale[r] = 1 / |w| (0 for a zero vector).
__global__ __launch_bounds__(kBlock) void k_arnoldi_col(int nv, int ld, const Z* __restrict__ h1,
                                                         const Z* __restrict__ n1, const Z* __restrict__ h2,
                                                         const Z* __restrict__ n2, const int* __restrict__ gate,
                                                         Z* __restrict__ col, double* __restrict__ scale,
                                                         const int* __restrict__ jd) {
  const int r = blockIdx.x;
  const int g = gate[r];
  if (jd) nv = *jd + 1;
  for (int i = threadIdx.x; i < nv; i += kBlock) {
    const Z a = h1[(size_t)r * ld + i];
    const Z b = g ? h2[(size_t)r * ld + i] : Z{0, 0};
    col[(size_t)r * ld + i] = Z{a.x + b.x, a.y + b.y};
  }
  if (threadIdx.x == 0) {
    const double nn = sqrt(fmax(0.0, g ? n2[r].x : n1[r].x));
    col[(size_t)r * ld + nv] = Z{nn, 0};
    col[(size_t)r * ld + nv + 1] = Z{(double)g, 0};
    scale[r] = nn > 0 ? 1.0 / nn : 0.0;
  }
}

// out[r] = a[r] * s[r] with a real per-RHS factor (rounded to the basis
// precision); conv (if not null) receives the same rounded values in the
// product's precision D, the input of the next product.  With jd (the
// Arnoldi step index on the device), out is V_{*jd + 1} of the basis at out.
template <typename VB, typename D>
__global__ __launch_bounds__(kBlock) void k_scale_real(size_t Nt, const Z* __restrict__ a,
                                                        const double* __restrict__ s, C2<VB>* __restrict__ out,
                                                        C2<D>* __restrict__ conv, size_t vstride,
                                                        const int* __restrict__ jd) {
  const int r = blockIdx.y;
  const double c = s[r];
  if (jd) out += (size_t)(*jd + 1) * vstride;
  for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < Nt; k += (size_t)gridDim.x * kBlock) {
    const Z v = a[(size_t)r * Nt + k];
    const C2<VB> q{(VB)(v.x * c), (VB)(v.y * c)};
    out[(size_t)r * Nt + k] = q;
    if (conv) conv[(size_t)r * Nt + k] = C2<D>{(D)q.x, (D)q.y};
  }
}
__global__ void k_set_step(int* __restrict__ jd, int v, int add) {
  if (threadIdx.x == 0) jd[0] = add ? jd[0] + v : v;
}

// out += a
__global__ __launch_bounds__(kBlock) void k_add(size_t cnt, const Z* __restrict__ a, Z* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < cnt; i += (size_t)gridDim.x * kBlock)
    out[i] = {out[i].x + a[i].x, out[i].y + a[i].y};
}

// out = a - b
__global__ __launch_bounds__(kBlock) void k_sub(size_t cnt, const Z* __restrict__ a, const Z* __restrict__ b, Z* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < cnt; i += (size_t)gridDim.x * kBlock)
    out[i] = {a[i].x - b[i].x, a[i].y - b[i].y};
}

// out[r] = sum_i V[i][r] y[r][i] (+ out if accumulate)
template <typename VB>
__global__ __launch_bounds__(kBlock) void k_combine(int nv, int ld_r, size_t Nt, size_t vstride, const C2<VB>* __restrict__ V,
                                                     const Z* __restrict__ yv, Z* __restrict__ out, int accumulate) {
  const int r = blockIdx.y;
  for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < Nt; k += (size_t)gridDim.x * kBlock) {
    Z acc = accumulate ? out[(size_t)r * Nt + k] : Z{0, 0};
    for (int i = 0; i < nv; ++i) {
      const C2<VB> t = V[i * vstride + (size_t)r * Nt + k];
      const Z v{(double)t.x, (double)t.y};
      const Z c = yv[(size_t)r * ld_r + i];
      acc.x += v.x * c.x - v.y * c.y;
      acc.y += v.x * c.y + v.y * c.x;
    }
    out[(size_t)r * Nt + k] = acc;
  }
}

// --------------------------------------------------------------- buffers --
struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevMem& operator=(DevMem&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevMem() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t b) {
    release();
    if (b == 0) return hipSuccess;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) bytes = b;
    return e;
  }
  template <typename U>
  U* as() const { return reinterpret_cast<U*>(p); }
};

// Pinned host staging for the small per-iteration GMRES transfers.
struct HostMem {
  void* p = nullptr;
  size_t bytes = 0;
  HostMem() = default;
  HostMem(const HostMem&) = delete;
  HostMem& operator=(const HostMem&) = delete;
  ~HostMem() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t b) {
    if (b <= bytes) return hipSuccess;
    release();
    hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
    if (e == hipSuccess) bytes = b;
    return e;
  }
  template <typename U>
  U* as() const { return reinterpret_cast<U*>(p); }
};

int grid1d(size_t work) {
  size_t b = (work + kBlock - 1) / kBlock;
  return (int)std::max<size_t>(1, std::min<size_t>(b, 65535));
}

template <typename T>
class EngineT final : public Engine {
  using CT = C2<T>;
  struct Pending {  // a profiled stage whose launch has not happened yet
    int stage = -1;
    hipEvent_t a = nullptr, b = nullptr;
  };
  struct Lvl {
    int nx, ny, nt, np, K;
    DevMem TL, TLp;  // TLp: FP32 only, the far offsets' operators in pairs
    DevMem il_cnt, il_src, il_off;  // interaction lists
    DevMem S, G;  // pattern buffers, sized for R_alloc
  };
  // One level's streamed interpolation plan (aggregation into this level,
  // disaggregation out of it): stencil tables, windows and row chunks.  The
  // row chunks are tabulated for a few batch sizes (kChunkR), since a larger
  // batch needs fewer chunks to fill the chip.
  struct Itp {
    int order = 0;
    int a_nst = 0, a_wlen = 0, d_nst = 0, d_wlen = 0, d_ntap = 0;
    int a_sw = kIStrip, d_sw = kIStrip;         // strip widths (16: two components per wave)
    int a_ends = 3;                              // most parent rows ending at one extended child row
    int a_rows = 0, d_rows = 0;                 // rows per chunk set by the tuner (0: planner)
    int a_nch[8] = {}, d_nch[8] = {};           // chunks per batch-size bucket
    int a_coff[8] = {}, d_coff[8] = {};         // offsets of the buckets' chunk tables
    DevMem s0, vrow, vflip, thw_a, thw_d, colb_a, colw_a, colb_d, colw_d, wlo_a, wlo_d, E;
    DevMem chunk_a, chunk_d, chunkp_d;
  };
  static constexpr int kChunkR[8] = {1, 2, 4, 8, 16, 32, 64, 1 << 30};
  static int chunk_bucket(int R) {
    int b = 0;
    while (b < 7 && kChunkR[b] < R) ++b;
    return b;
  }

 public:
  int upload(const Upload& u, std::string& err) override {
    N_ = u.N;
    n_ = u.n;
    P_ = u.P;
    nc_ = u.n_classes;
    const Tree& tr = *u.tree;
    tree_ = u.tree;
    ntl_ = tr.ntl;
    if (ntl_ > kMaxTrLv) {
      err = "more than " + std::to_string(kMaxTrLv) + " tree levels";
      return -1;
    }
    lv_.clear();
    lv_.resize(ntl_);
    it_.clear();
    it_.resize(std::max(ntl_, 1));
    for (int l = 0; l < ntl_; ++l) {
      const LevelGrid& g = tr.lv[l];
      Lvl& L = lv_[l];
      L.nx = g.nx;
      L.ny = g.ny;
      L.nt = g.nt;
      L.np = g.np;
      L.K = g.K;
      if (int rc = put_c(L.TL, tr.TL[l], err)) return rc;
      if constexpr (std::is_same<T, float>::value) {
        std::vector<cd> tlp((size_t)40 * L.K);
        for (int q = 0; q < 20; ++q)
          for (int s2 = 0; s2 < L.K; ++s2)
            for (int h = 0; h < 2; ++h)
              tlp[((size_t)q * L.K + s2) * 2 + h] = tr.TL[l][(size_t)tr_far_offset(2 * q + h) * L.K + s2];
        if (int rc = put_c(L.TLp, tlp, err)) return rc;
      }
      // interaction lists: children of the parent's neighbours that are not
      // neighbours themselves
      std::vector<int> cnt(L.nx * L.ny, 0), src((size_t)L.nx * L.ny * kMaxIL, 0), off((size_t)L.nx * L.ny * kMaxIL, 0);
      for (int J = 0; J < L.ny; ++J)
        for (int I = 0; I < L.nx; ++I) {
          const int p = J * L.nx + I;
          for (int dy = -3; dy <= 3; ++dy)
            for (int dx = -3; dx <= 3; ++dx) {
              if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
              const int I2 = I + dx, J2 = J + dy;
              if (I2 < 0 || J2 < 0 || I2 >= L.nx || J2 >= L.ny) continue;
              if (std::abs((I2 >> 1) - (I >> 1)) > 1 || std::abs((J2 >> 1) - (J >> 1)) > 1) continue;
              src[(size_t)p * kMaxIL + cnt[p]] = J2 * L.nx + I2;
              off[(size_t)p * kMaxIL + cnt[p]] = (dy + 3) * 7 + (dx + 3);
              cnt[p]++;
            }
        }
      if (int rc = put_i(L.il_cnt, cnt, err)) return rc;
      if (int rc = put_i(L.il_src, src, err)) return rc;
      if (int rc = put_i(L.il_off, off, err)) return rc;
    }
    for (int l = 1; l < ntl_; ++l)
      if (int rc = plan_level(l, 0, 0, err)) return rc;
    // leaf data
    nx0_ = u.nx0;
    ny0_ = u.ny0;
    if (int rc = put_i(box_of_, u.box_of, err)) return rc;
    // field evaluation: particle centres, and the leaf sphere's directions,
    // unit vectors and weights [K0][khat, th_hat, ph_hat, w]
    fld_k_ = u.k;
    fld_L_ = ntl_ > 0 ? tr.lv[0].L : 0;
    {
      std::vector<double> cen((size_t)P_ * 3);
      for (int p = 0; p < P_; ++p) {
        cen[3 * p] = u.centers[p].x;
        cen[3 * p + 1] = u.centers[p].y;
        cen[3 * p + 2] = u.centers[p].z;
      }
      if (int rc = put_raw(fld_cen_, cen.data(), cen.size(), err)) return rc;
      if (ntl_ > 0) {
        const LevelGrid& g = tr.lv[0];
        std::vector<float> tab((size_t)g.K * 10);
        for (int s = 0; s < g.K; ++s) {
          const V3 v[3] = {g.khat[s], g.th_hat[s], g.ph_hat[s]};
          for (int c = 0; c < 3; ++c) {
            tab[(size_t)s * 10 + 3 * c] = (float)v[c].x;
            tab[(size_t)s * 10 + 3 * c + 1] = (float)v[c].y;
            tab[(size_t)s * 10 + 3 * c + 2] = (float)v[c].z;
          }
          tab[(size_t)s * 10 + 9] = (float)g.w[s];
        }
        if (int rc = put_raw(fld_tab_, tab.data(), tab.size(), err)) return rc;
      }
    }
    if (int rc = put_i(class_of_, u.class_of, err)) return rc;
    if (int rc = put_i(order_, u.order, err)) return rc;
    if (int rc = put_i(tile_start_, u.tile_start, err)) return rc;
    if (int rc = put_i(tile_count_, u.tile_count, err)) return rc;
    if (int rc = put_i(tile_class_, u.tile_class, err)) return rc;
    ntiles_ = (int)u.tile_start.size();
    tp_ = u.tile_count.empty() ? 0 : *std::max_element(u.tile_count.begin(), u.tile_count.end());
    M2_ = ntl_ > 0 ? 2 * lv_[0].K : 0;
    {
      std::vector<cd> rm, qm;
      std::vector<int> ro, qo;
      for (int c = 0; c < nc_; ++c) {
        ro.push_back((int)rm.size());
        qo.push_back((int)qm.size());
        rm.insert(rm.end(), u.Rm[c].begin(), u.Rm[c].end());
        qm.insert(qm.end(), u.Qm[c].begin(), u.Qm[c].end());
      }
      if (int rc = put_c(Rm_, rm, err)) return rc;
      if (int rc = put_c(Qm_, qm, err)) return rc;
      if (int rc = put_i(rm_off_, ro, err)) return rc;
      if (int rc = put_i(qm_off_, qo, err)) return rc;
    }
    {
      std::vector<cd> all;
      for (auto& m : u.near_mats) all.insert(all.end(), m.begin(), m.end());
      if (int rc = put_c(near_mats_, all, err)) return rc;
      if (int rc = put_i(near_nbr_, u.near_nbr, err)) return rc;
      if (int rc = put_i(near_slot_, u.near_slot, err)) return rc;
      std::vector<cd> zi;
      for (auto& m : u.Zinv) zi.insert(zi.end(), m.begin(), m.end());
      if (int rc = put_c(zinv_, zi, err)) return rc;
      std::vector<int> self_nbr(P_), self_slot(P_);
      for (int p = 0; p < P_; ++p) {
        self_nbr[p] = p;
        self_slot[p] = u.class_of[p];
      }
      if (int rc = put_i(self_nbr_, self_nbr, err)) return rc;
      if (int rc = put_i(self_slot_, self_slot, err)) return rc;
      // per particle tile and slot: the shared matrix, -1 (none) or -2 (mixed)
      auto tile_slots = [&](const std::vector<int>& nbr, const std::vector<int>& slot, int nsp) {
        const int ntl = (P_ + kTPN - 1) / kTPN;
        std::vector<int> ts((size_t)ntl * nsp, -1);
        for (int t = 0; t < ntl; ++t)
          for (int o = 0; o < nsp; ++o) {
            int v = -1;
            for (int p = t * kTPN; p < std::min(P_, (t + 1) * kTPN); ++p) {
              if (nbr[(size_t)p * nsp + o] < 0) continue;
              const int sl = slot[(size_t)p * nsp + o];
              v = (v == -1 || v == sl) ? sl : -2;
            }
            ts[(size_t)t * nsp + o] = v;
          }
        return ts;
      };
      if (int rc = put_i(near_tile_slot_, tile_slots(u.near_nbr, u.near_slot, 9), err)) return rc;
      if (int rc = put_i(self_tile_slot_, tile_slots(self_nbr, self_slot, 1), err)) return rc;
    }
    centers_ = u.centers;
    nslots_ = (int)u.near_mats.size();
    nnear_ = 0;
    for (int q : u.near_nbr) nnear_ += q >= 0;
    pairs_.assign(ntl_, 0);
    for (int l = 0; l < ntl_; ++l) {
      const Lvl& L = lv_[l];
      for (int J = 0; J < L.ny; ++J)
        for (int I = 0; I < L.nx; ++I)
          for (int dy = -3; dy <= 3; ++dy)
            for (int dx = -3; dx <= 3; ++dx) {
              if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
              const int I2 = I + dx, J2 = J + dy;
              if (I2 < 0 || J2 < 0 || I2 >= L.nx || J2 >= L.ny) continue;
              if (std::abs((I2 >> 1) - (I >> 1)) > 1 || std::abs((J2 >> 1) - (J >> 1)) > 1) continue;
              pairs_[l]++;
            }
    }
    if (int rc = upload_mfma(u, err)) return rc;
    R_alloc_ = 0;
    return 0;
  }

  // Real 2x2-block forms of the dense contractions for the matrix cores
  // (FP32 contexts only): radiation and receiving matrices per class, and
  // the nine near blocks side by side when every particle uses the same
  // block for a given neighbour offset.
  int upload_mfma(const Upload& u, std::string& err) {
    mfma_ = std::is_same<T, float>::value && std::getenv("MLFMA_NO_MFMA") == nullptr;
    bf16_ = mfma_ && u.precision == 2;
    near_uniform_ = false;
    if (!mfma_) return 0;
    const int n = n_, nf = 2 * n_;
    auto put_f = [&](DevMem& d, const std::vector<float>& v) { return put_raw(d, v.data(), v.size(), err); };
    // the BF16 heads and remainders of a matrix (round to nearest, ties to even)
    auto put_split = [&](DevMem& dh, DevMem& dl, const std::vector<float>& v) -> int {
      if (!bf16_) return 0;
      auto tobf = [](float f) {
        uint32_t u;
        std::memcpy(&u, &f, 4);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
      };
      std::vector<uint16_t> h(v.size()), l(v.size());
      for (size_t i = 0; i < v.size(); ++i) {
        h[i] = tobf(v[i]);
        const uint32_t hb = (uint32_t)h[i] << 16;
        float hf;
        std::memcpy(&hf, &hb, 4);
        l[i] = tobf(v[i] - hf);
      }
      if (int rc = put_raw(dh, h.data(), h.size(), err)) return rc;
      return put_raw(dl, l.data(), l.size(), err);
    };
    auto block2 = [](std::vector<float>& A, size_t lda, size_t row, size_t col, cd z) {
      A[row * lda + col] = (float)z.real();
      A[row * lda + col + 1] = (float)-z.imag();
      A[(row + 1) * lda + col] = (float)z.imag();
      A[(row + 1) * lda + col + 1] = (float)z.real();
    };
    // GEMM columns of the projection and receive: particles grouped by class
    // (the class-sorted order), each class padded to whole 16-column tiles
    // (padding columns are -1: zero input, not written); one matrix offset
    // per column tile.
    {
      std::vector<int> part, box, aop, aor, aoz;
      const int nf0 = 2 * n_;
      size_t i = 0;
      while (i < u.order.size()) {
        const int c = u.class_of[u.order[i]];
        size_t e = i;
        while (e < u.order.size() && u.class_of[u.order[e]] == c) ++e;
        for (size_t k = i; k < e; ++k) {
          part.push_back(u.order[k]);
          box.push_back(u.box_of[u.order[k]]);
        }
        while (part.size() % 16) {
          part.push_back(-1);
          box.push_back(-1);
        }
        while (aop.size() < part.size() / 16) {
          aop.push_back(c * 2 * M2_ * nf0);
          aor.push_back(c * nf0 * 2 * M2_);
          aoz.push_back(c * nf0 * nf0);
        }
        i = e;
      }
      ncols_pad_ = (int)part.size();
      if (int rc = put_i(gcol_part_, part, err)) return rc;
      if (int rc = put_i(gcol_box_, box, err)) return rc;
      if (int rc = put_i(a_off_proj_, aop, err)) return rc;
      if (int rc = put_i(a_off_recv_, aor, err)) return rc;
      if (int rc = put_i(a_off_zinv_, aoz, err)) return rc;
      // inverse self blocks of the classes (the block-diagonal preconditioner)
      std::vector<float> Az((size_t)nc_ * nf0 * nf0, 0.f);
      for (int c = 0; c < nc_; ++c) {
        const cd* Zt = u.Zinv[c].data();  // transposed: [k][j]
        std::vector<float> a((size_t)nf0 * nf0, 0.f);
        for (int j2 = 0; j2 < n; ++j2)
          for (int k2 = 0; k2 < n; ++k2) block2(a, nf0, 2 * j2, 2 * k2, Zt[(size_t)k2 * n + j2]);
        std::copy(a.begin(), a.end(), Az.begin() + (size_t)c * a.size());
      }
      if (int rc = put_f(A_zinv_, Az)) return rc;
    }
    if (ntl_ > 0) {
      const int M2 = M2_;
      std::vector<float> Ap((size_t)nc_ * 2 * M2 * nf, 0.f), Ar((size_t)nc_ * nf * 2 * M2, 0.f);
      for (int c = 0; c < nc_; ++c) {
        const cd* R = u.Rm[c].data();  // [j][mc]
        const cd* Q = u.Qm[c].data();  // [mc][j]
        std::vector<float> a((size_t)2 * M2 * nf, 0.f), b((size_t)nf * 2 * M2, 0.f);
        for (int mc = 0; mc < M2; ++mc)
          for (int j = 0; j < n; ++j) {
            block2(a, nf, 2 * mc, 2 * j, R[(size_t)j * M2 + mc]);
            block2(b, 2 * M2, 2 * j, 2 * mc, Q[(size_t)mc * n + j]);
          }
        std::copy(a.begin(), a.end(), Ap.begin() + (size_t)c * a.size());
        std::copy(b.begin(), b.end(), Ar.begin() + (size_t)c * b.size());
      }
      if (int rc = put_f(A_proj_, Ap)) return rc;
      if (int rc = put_f(A_recv_, Ar)) return rc;
      if (int rc = put_split(A_proj_h_, A_proj_l_, Ap)) return rc;
      if (int rc = put_split(A_recv_h_, A_recv_l_, Ar)) return rc;
    }
    // near blocks: one matrix per offset shared by all particles?
    std::vector<int> sl(9, -1);
    bool uniform = true;
    for (int p = 0; p < P_ && uniform; ++p)
      for (int o = 0; o < 9; ++o) {
        if (u.near_nbr[(size_t)p * 9 + o] < 0) continue;
        const int sv = u.near_slot[(size_t)p * 9 + o];
        if (sl[o] == -1) sl[o] = sv;
        else if (sl[o] != sv) uniform = false;
      }
    near_uniform_ = uniform;
    if (uniform) {
      const size_t lda = (size_t)9 * nf;
      std::vector<float> An((size_t)nf * lda, 0.f);
      for (int o = 0; o < 9; ++o) {
        if (sl[o] < 0) continue;
        const cd* Zt = u.near_mats[sl[o]].data();  // transposed: [k][j] = Z[j][k]
        for (int j = 0; j < n; ++j)
          for (int k = 0; k < n; ++k) block2(An, lda, 2 * j, (size_t)o * nf + 2 * k, Zt[(size_t)k * n + j]);
      }
      if (int rc = put_f(A_near_, An)) return rc;
      if (int rc = put_split(A_near_h_, A_near_l_, An)) return rc;
      std::vector<int> iota(P_);
      for (int p = 0; p < P_; ++p) iota[p] = p;
      if (int rc = put_i(iota_, iota, err)) return rc;
    } else {
      // class-pair blocks differ between particles: one GEMM column per
      // (particle, neighbour) pair, grouped by block (slot) and padded to
      // whole 16-column tiles, each tile multiplying its slot's matrix; the
      // products land in partial[(o * P + p)] and k_near_sum adds the nine.
      const int ns = (int)u.near_mats.size();
      std::vector<float> Aall((size_t)ns * nf * nf, 0.f);
      for (int sl2 = 0; sl2 < ns; ++sl2) {
        const cd* Zt = u.near_mats[sl2].data();
        std::vector<float> a((size_t)nf * nf, 0.f);
        for (int j = 0; j < n; ++j)
          for (int k = 0; k < n; ++k) block2(a, nf, 2 * j, 2 * k, Zt[(size_t)k * n + j]);
        std::copy(a.begin(), a.end(), Aall.begin() + (size_t)sl2 * nf * nf);
      }
      std::vector<std::vector<std::pair<int, int>>> by_slot(ns);  // (neighbour q, o * P + p)
      for (int p = 0; p < P_; ++p)
        for (int o = 0; o < 9; ++o) {
          const int q = u.near_nbr[(size_t)p * 9 + o];
          if (q >= 0) by_slot[u.near_slot[(size_t)p * 9 + o]].push_back({q, o * P_ + p});
        }
      std::vector<int> bq, cq, aoff;
      for (int sl2 = 0; sl2 < ns; ++sl2) {
        if (by_slot[sl2].empty()) continue;
        for (auto& e : by_slot[sl2]) {
          bq.push_back(e.first);
          cq.push_back(e.second);
        }
        while (bq.size() % 16) {
          bq.push_back(-1);
          cq.push_back(-1);
        }
        while (aoff.size() < bq.size() / 16) aoff.push_back(sl2 * nf * nf);
      }
      ngcols_ = (int)bq.size();
      if (int rc = put_f(A_near_, Aall)) return rc;
      if (int rc = put_split(A_near_h_, A_near_l_, Aall)) return rc;
      if (int rc = put_i(ng_bcol_, bq, err)) return rc;
      if (int rc = put_i(ng_ccol_, cq, err)) return rc;
      if (int rc = put_i(ng_aoff_, aoff, err)) return rc;
      std::vector<int> has((size_t)P_ * 9);
      for (size_t i = 0; i < has.size(); ++i) has[i] = u.near_nbr[i] >= 0;
      if (int rc = put_i(ng_has_, has, err)) return rc;
    }
    return 0;
  }

  // Streamed interpolation plan of level l (parent) and l - 1 (child):
  // tables and, for each batch-size bucket, row chunks so that a launch has
  // about kStreamItems waves.  agg_rows: parent rows per aggregation chunk,
  // dis_rows: extended child rows per disaggregation chunk (0: planner).
  // Chunking changes only which wave computes an output, not its arithmetic.
  int plan_level(int l, int agg_rows, int dis_rows, std::string& err) {
    const Lvl &C = lv_[l - 1], &Pp = lv_[l];
    const LevelGrid &gc = tree_->lv[l - 1], &gp = tree_->lv[l];
    const InterpTables& T0 = tree_->it[l];
    Itp& I = it_[l];
    const int ORD = T0.order, nvr = C.nt + ORD;
    I.order = ORD;
    if (C.np % 2 || Pp.np % 2 || (int)T0.vrow.size() != nvr) {
      err = "interpolation: odd phi sample counts at level " + std::to_string(l);
      return -1;
    }
    // the streamed kernels address one RHS's patterns of a level with 32-bit
    // byte offsets
    for (const Lvl* V : {&C, &Pp})
      if ((double)V->nx * V->ny * 2.0 * V->K * sizeof(C2<T>) >= 4294967296.0) {
        err = "interpolation: one RHS's patterns exceed 4 GiB at level " + std::to_string(l);
        return -1;
      }
    // theta: the stencils on the extended rows must be the recorded taps
    for (int p = 0; p < Pp.nt; ++p)
      for (int a = 0; a < ORD; ++a) {
        const int e = T0.th_s0[p] + a;
        if (e < 0 || e >= nvr || T0.vrow[e] != T0.th_row[(size_t)p * ORD + a] ||
            T0.vflip[e] != T0.th_flip[(size_t)p * ORD + a] || (p > 0 && T0.th_s0[p] < T0.th_s0[p - 1])) {
          err = "interpolation: theta stencils are not runs of extended rows at level " + std::to_string(l);
          return -1;
        }
      }
    {
      std::vector<int> ends(nvr, 0);
      I.a_ends = 1;
      for (int p = 0; p < Pp.nt; ++p) {
        if (++ends[T0.th_s0[p] + ORD - 1] > 3) {
          err = "interpolation: more than 3 parent rows end at one child row at level " + std::to_string(l);
          return -1;
        }
        I.a_ends = std::max(I.a_ends, ends[T0.th_s0[p] + ORD - 1]);
      }
      if (C.nt < ORD) {
        err = "interpolation: fewer child rows than stencil points at level " + std::to_string(l);
        return -1;
      }
    }
    std::vector<double> thw_d((size_t)Pp.nt * ORD);
    for (int p = 0; p < Pp.nt; ++p)
      for (int a = 0; a < ORD; ++a)
        thw_d[(size_t)p * ORD + a] =
            T0.th_w[(size_t)p * ORD + a] * gp.wtheta[p] / gc.wtheta[T0.vrow[T0.th_s0[p] + a]];
    // phi, forward: each parent column reads ORD consecutive child columns
    std::vector<int> colb_a(Pp.np);
    for (int j = 0; j < Pp.np; ++j) {
      colb_a[j] = T0.ph_col[(size_t)j * ORD];
      for (int b = 0; b < ORD; ++b)
        if (T0.ph_col[(size_t)j * ORD + b] != (colb_a[j] + b) % C.np) {
          err = "interpolation: phi stencil is not a run of columns at level " + std::to_string(l);
          return -1;
        }
    }
    // phi, transposed: each child column gathers the cyclic run of parent
    // columns whose stencils contain it (a weight may be exactly zero where
    // a parent node falls on a child node), weight times np_c / np_p
    std::vector<std::vector<double>> dense((size_t)C.np, std::vector<double>(Pp.np, 0.0));
    std::vector<std::vector<char>> member((size_t)C.np, std::vector<char>(Pp.np, 0));
    for (int j = 0; j < Pp.np; ++j)
      for (int b = 0; b < ORD; ++b) {
        dense[(colb_a[j] + b) % C.np][j] += T0.ph_w[(size_t)j * ORD + b];
        member[(colb_a[j] + b) % C.np][j] = 1;
      }
    std::vector<int> colb_d(C.np), cnt_d(C.np);
    int ntap = 0;
    for (int c = 0; c < C.np; ++c) {
      int first = -1, cnt = 0;
      for (int j = 0; j < Pp.np; ++j)
        if (member[c][j]) {
          ++cnt;
          if (!member[c][(j + Pp.np - 1) % Pp.np]) first = j;
        }
      if (first < 0 || cnt == Pp.np) {
        err = "interpolation: transposed phi stencil is not a run at level " + std::to_string(l);
        return -1;
      }
      for (int k = 0; k < cnt; ++k)
        if (!member[c][(first + k) % Pp.np]) {
          err = "interpolation: transposed phi stencil has a gap at level " + std::to_string(l);
          return -1;
        }
      colb_d[c] = first;
      cnt_d[c] = cnt;
      ntap = std::max(ntap, cnt);
    }
    // (10 taps, the finest levels' count with 6-point stencils, only with those)
    ntap = ntap <= 8 ? 8 : ntap <= 10 && ORD == 6 ? 10 : ntap <= 12 ? 12 : ntap <= 16 ? 16 : -1;
    if (ntap < 0) {
      err = "interpolation: more than 16 transposed phi taps at level " + std::to_string(l);
      return -1;
    }
    std::vector<double> colw_d((size_t)C.np * ntap, 0.0);
    for (int c = 0; c < C.np; ++c)
      for (int k = 0; k < cnt_d[c]; ++k)
        colw_d[(size_t)c * ntap + k] = dense[c][(colb_d[c] + k) % Pp.np] * (double)C.np / (double)Pp.np;
    // windows of the half-waves: strips of sw output columns (16 where half a
    // row fits, so that a wave takes both components)
    // (pairs: windows start at even columns and have even lengths, for the
    // aggregation's paired staging loads on 32-column strips)
    auto windows = [](int nout, int nin, const std::vector<int>& colb, int taps, std::vector<int>& wlo, int& nst,
                      int& sw, bool pairs) {
      const int ho = nout / 2;
      sw = ho <= kIStrip / 2 ? kIStrip / 2 : kIStrip;
      pairs = pairs && sw == kIStrip;
      nst = (ho + sw - 1) / sw;
      wlo.assign((size_t)2 * nst, 0);
      int wl = 0;
      for (int st = 0; st < nst; ++st)
        for (int h = 0; h < 2; ++h) {
          const int j0 = st * sw + h * ho, j1 = std::min(st * sw + sw, ho) - 1 + h * ho;
          const int w0 = pairs ? colb[j0] & ~1 : colb[j0];
          wlo[(size_t)st * 2 + h] = w0;
          wl = std::max(wl, (colb[j1] - w0 + nin) % nin + taps);
        }
      return pairs ? wl + (wl & 1) : wl;
    };
    std::vector<int> wlo_a, wlo_d;
    I.a_wlen = windows(Pp.np, C.np, colb_a, ORD, wlo_a, I.a_nst, I.a_sw, true);
    I.d_wlen = windows(C.np, Pp.np, colb_d, ntap, wlo_d, I.d_nst, I.d_sw, false);
    I.d_ntap = ntap;
    // staged values per lane and row: the aggregation's four children (4, or
    // 6 with two components per wave), the disaggregation's parent (3)
    const int ks_a = I.a_sw == kIStrip ? kIStage / 2 : 3 * kIStage / 4, ks_d = 3 * kIStage / 8;
    if ((kIStrip / I.a_sw) * 8 * I.a_wlen > 64 * ks_a || (kIStrip / I.d_sw) * 2 * I.d_wlen > 64 * ks_d) {
      err = "interpolation: phi windows too wide at level " + std::to_string(l);
      return -1;
    }
    // chunks per batch-size bucket
    I.a_rows = agg_rows;
    I.d_rows = dis_rows;
    std::vector<int> ca, cdv, cpd;
    const size_t nbp = (size_t)Pp.nx * Pp.ny;
    for (int b = 0; b < 8; ++b) {
      const size_t Rb = (size_t)std::min(kChunkR[b], 64);
      // aggregation: chunks of parent rows
      const size_t base_a = Rb * nbp * (I.a_sw == kIStrip ? 2 : 1) * I.a_nst;
      int na = agg_rows > 0 ? (Pp.nt + agg_rows - 1) / agg_rows
                            : (int)std::min<size_t>((kStreamItems + base_a - 1) / base_a,
                                                    (size_t)std::max(1, Pp.nt / (2 * ORD)));
      na = std::max(1, std::min(na, Pp.nt));
      I.a_nch[b] = na;
      I.a_coff[b] = (int)ca.size();
      for (int i = 0; i <= na; ++i) ca.push_back((int)((long long)i * Pp.nt / na));
      // disaggregation: chunks of extended child rows; interior cuts in
      // [ORD, nt_c] so that a pole reflection stays with its row
      const size_t base_d = Rb * nbp * (I.d_sw == kIStrip ? 2 : 1) * I.d_nst;
      const int span = C.nt - ORD;
      int nd = dis_rows > 0 ? (nvr + dis_rows - 1) / dis_rows
                            : (int)std::min<size_t>((kStreamItems + base_d - 1) / base_d,
                                                    (size_t)std::max(1, C.nt / (2 * ORD)));
      nd = span <= 0 ? 1 : std::max(1, std::min(nd, span + 1));
      I.d_nch[b] = nd;
      I.d_coff[b] = (int)cdv.size();
      cdv.push_back(0);
      for (int i = 1; i < nd; ++i) cdv.push_back(ORD + (int)((long long)i * span / nd));
      cdv.push_back(nvr);
      for (int i = 0; i < nd; ++i) {
        const int E0 = cdv[I.d_coff[b] + i], E1 = cdv[I.d_coff[b] + i + 1];
        int pf = -1, pl = -1;
        for (int p = 0; p < Pp.nt; ++p) {
          if (pf < 0 && T0.th_s0[p] + ORD - 1 >= E0) pf = p;
          if (T0.th_s0[p] <= E1 - 1) pl = p;
        }
        if (pf < 0 || pl < pf) {
          err = "interpolation: empty disaggregation chunk at level " + std::to_string(l);
          return -1;
        }
        cpd.push_back(pf);
        cpd.push_back(pl);
      }
    }
    std::vector<int> vflip(T0.vflip.begin(), T0.vflip.end());
    std::vector<cd> E((size_t)2 * Pp.K);  // pairs, one per parent sample
    for (int s2 = 0; s2 < Pp.K; ++s2) {
      E[(size_t)2 * s2] = T0.phase[(size_t)3 * Pp.K + s2];      // child offset (+a/2, +a/2)
      E[(size_t)2 * s2 + 1] = T0.phase[(size_t)1 * Pp.K + s2];  // (+a/2, -a/2)
    }
    if (int rc = put_i(I.s0, T0.th_s0, err)) return rc;
    if (int rc = put_i(I.vrow, T0.vrow, err)) return rc;
    if (int rc = put_i(I.vflip, vflip, err)) return rc;
    if (int rc = put_r(I.thw_a, T0.th_w, err)) return rc;
    if (int rc = put_r(I.thw_d, thw_d, err)) return rc;
    if (int rc = put_i(I.colb_a, colb_a, err)) return rc;
    if (int rc = put_r(I.colw_a, T0.ph_w, err)) return rc;
    if (int rc = put_i(I.colb_d, colb_d, err)) return rc;
    if (int rc = put_r(I.colw_d, colw_d, err)) return rc;
    if (int rc = put_i(I.wlo_a, wlo_a, err)) return rc;
    if (int rc = put_i(I.wlo_d, wlo_d, err)) return rc;
    if (int rc = put_c(I.E, E, err)) return rc;
    if (int rc = put_i(I.chunk_a, ca, err)) return rc;
    if (int rc = put_i(I.chunk_d, cdv, err)) return rc;
    if (int rc = put_i(I.chunkp_d, cpd, err)) return rc;
    return 0;
  }

  // All levels or none: on a tile that does not fit, the previous plan is
  // restored.
  int set_gemm_tiles(int rt_np, int rt_recv, std::string& err) override {
    auto ok = [](int v) { return v == 0 || v == 1 || v == 2 || v == 4; };
    if (!ok(rt_np) || !ok(rt_recv)) {
      err = "GEMM row tiles must be 1, 2 or 4 (0: default 4)";
      return -1;
    }
    rt_np_ = rt_np ? rt_np : 4;
    rt_recv_ = rt_recv ? rt_recv : 4;
    clear_graphs();
    return 0;
  }
  void get_gemm_tiles(int& rt_np, int& rt_recv) const override {
    rt_np = rt_np_;
    rt_recv = rt_recv_;
  }

  int set_tuning(const std::vector<int>& agg_rows, const std::vector<int>& dis_rows, std::string& err) override {
    for (int v : agg_rows)
      if (v < 0) {
        err = "row chunks must be >= 0 (0: planner)";
        return -1;
      }
    for (int v : dis_rows)
      if (v < 0) {
        err = "row chunks must be >= 0 (0: planner)";
        return -1;
      }
    std::vector<int> pa, pd;
    get_tuning(pa, pd);
    clear_graphs();
    for (int l = 1; l < ntl_; ++l) {
      const int a = l < (int)agg_rows.size() ? agg_rows[l] : 0;
      const int d = l - 1 < (int)dis_rows.size() ? dis_rows[l - 1] : 0;
      if (int rc = plan_level(l, a, d, err)) {
        std::string ignored;
        for (int k = 1; k < ntl_; ++k) (void)plan_level(k, pa[k], pd[k - 1], ignored);
        return rc;
      }
    }
    return 0;
  }

  void get_tuning(std::vector<int>& agg_rows, std::vector<int>& dis_rows) const override {
    agg_rows.assign(std::max(ntl_, 1), 0);
    dis_rows.assign(std::max(ntl_, 1), 0);
    for (int l = 1; l < ntl_; ++l) {
      agg_rows[l] = it_[l].a_rows;
      dis_rows[l - 1] = it_[l].d_rows;
    }
  }

  // near-field products of the class-pair GEMM: partial[r][o * P + p][:]
  GemmJob near_group_job(const CT* x, int rt) const {
    const int nf = 2 * n_;
    GemmJob j{};
    j.A = A_near_.template as<float>();
    j.Ah = A_near_h_.template as<unsigned short>();
    j.Al = A_near_l_.template as<unsigned short>();
    j.a_off = ng_aoff_.template as<int>();
    j.B = reinterpret_cast<const float*>(x);
    j.bcol = ng_bcol_.template as<int>();
    j.C = pNear_;
    j.ccol = ng_ccol_.template as<int>();
    j.sB = (size_t)P_ * nf;
    j.sC = (size_t)9 * P_ * nf;
    j.M = nf;
    j.ncols = ngcols_;
    j.nseg = 1;
    j.kseg = nf;
    j.lda = nf;
    j.ldb = nf;
    j.ldc = nf;
    j.acc = 0;
    j.tiles_m = (nf + 16 * rt - 1) / (16 * rt);
    j.tiles = j.tiles_m * (ngcols_ / 16);
    j.xcd = 1;  // consecutive tiles share a block matrix: keep them in one L2
    j.wtile = short_k(j);
    return j;
  }

  // The pattern buffers the product's kernels use: the context's own, or
  // the no-allocation entry point's static scratch.
  void bind_context_buffers() {
    for (int l = 0; l < ntl_; ++l) {
      pS_[l] = lv_[l].S.template as<CT>();
      pG_[l] = lv_[l].G.template as<CT>();
    }
    pNear_ = near_part_.template as<float>();
  }
  int ensure(int R, std::string& err) {
    bind_context_buffers();
    if (R <= R_alloc_) return 0;
    for (int l = 0; l < ntl_; ++l) {
      Lvl& L = lv_[l];
      const size_t bytes = (size_t)R * L.nx * L.ny * 2 * L.K * sizeof(CT);
      HIP_TRY(L.S.alloc(bytes));
      HIP_TRY(L.G.alloc(bytes));
      HIP_TRY(hipMemset(L.S.p, 0, bytes));  // empty leaf boxes stay zero
      HIP_TRY(hipMemset(L.G.p, 0, bytes));
    }
    if (mfma_ && !near_uniform_) HIP_TRY(near_part_.alloc((size_t)R * 9 * P_ * 2 * n_ * sizeof(float)));
    HIP_TRY(hipDeviceSynchronize());
    R_alloc_ = R;
    bind_context_buffers();
    return 0;
  }

  // Graph-cached product: the kernel sequence of one (x, y, R, parts)
  // combination is captured once on an internal stream and replayed on the
  // caller's stream.
  int matvec(const void* xv, void* yv, int R, int parts, void* stream, std::string& err) override {
    const int old_alloc = R_alloc_;
    if (int rc = ensure(R, err)) return rc;
    if (R_alloc_ != old_alloc) clear_graphs();
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!use_graphs_ || prof_on_) return enqueue(xv, yv, R, parts, st, err);
    GraphEntry* g = nullptr;
    for (auto& e : graphs_)
      if (e.x == xv && e.y == yv && e.R == R && e.parts == parts) g = &e;
    if (!g) {
      if (!cap_stream_) HIP_TRY(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
      if (graphs_.size() >= kMaxGraphs) {
        auto oldest = std::min_element(graphs_.begin(), graphs_.end(),
                                       [](const GraphEntry& a, const GraphEntry& b) { return a.used < b.used; });
        destroy_entry(*oldest);
        graphs_.erase(oldest);
      }
      GraphEntry e;
      e.x = xv;
      e.y = yv;
      e.R = R;
      e.parts = parts;
      HIP_TRY(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal));
      int rc = enqueue(xv, yv, R, parts, cap_stream_, err);
      hipGraph_t graph = nullptr;
      hipError_t ce = hipStreamEndCapture(cap_stream_, &graph);
      if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      HIP_TRY(ce);
      hipError_t ie = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIP_TRY(ie);
      graphs_.push_back(std::move(e));
      g = &graphs_.back();
    }
    g->used = ++use_clock_;
    HIP_TRY(hipGraphLaunch(g->exec, st));
    return 0;
  }

  // The product with the pattern buffers (and the class-pair near partials)
  // laid out in the static scratch: no allocation, no graph, direct
  // launches.  Fails with EINVAL if they need more than kScratchBytes.
  int matvec_noalloc(const void* xv, void* yv, int R, void* stream, std::string& err) override {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    size_t off = 0;
    size_t offS[kMaxTrLv] = {}, offG[kMaxTrLv] = {}, offN = 0;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off += (bytes + 255) / 256 * 256;
      return o;
    };
    for (int l = 0; l < ntl_; ++l) {
      const size_t bytes = (size_t)R * lv_[l].nx * lv_[l].ny * 2 * lv_[l].K * sizeof(CT);
      offS[l] = take(bytes);
      offG[l] = take(bytes);
    }
    if (mfma_ && !near_uniform_) offN = take((size_t)R * 9 * P_ * 2 * n_ * sizeof(float));
    if (off > kScratchBytes) {
      err = "matvec_noalloc: the product needs " + std::to_string(off) + " bytes of scratch for " +
            std::to_string(R) + " RHS, above the limit of " + std::to_string(kScratchBytes);
      return -1;
    }
    void* base = nullptr;
    if (int rc = scratch_address(&base, err)) return rc;
    unsigned char* b = static_cast<unsigned char*>(base);
    for (int l = 0; l < ntl_; ++l) {
      pS_[l] = reinterpret_cast<CT*>(b + offS[l]);
      pG_[l] = reinterpret_cast<CT*>(b + offG[l]);
    }
    pNear_ = reinterpret_cast<float*>(b + offN);
    // the leaf patterns of empty boxes must read zero: clear them with a
    // kernel (no memset node, should the caller capture this stream)
    if (ntl_ > 0) {
      const size_t cnt = (size_t)R * lv_[0].nx * lv_[0].ny * 2 * lv_[0].K;
      hipLaunchKernelGGL(k_fill_zero<T>, dim3(grid1d(cnt)), dim3(kBlock), 0, st, pS_[0], cnt);
    }
    const bool prof = prof_on_;
    prof_on_ = false;  // no per-stage events: their creation may allocate
    const int rc = enqueue(xv, yv, R, 3, st, err);
    prof_on_ = prof;
    bind_context_buffers();
    return rc;
  }

  // one wave per tile where K is short (at most 16 k-steps of 16) and B
  // columns are not segmented; the BF16-split kernel always splits K
  int short_k(const GemmJob& j) const { return !bf16_ && j.nseg == 1 && j.nseg * j.kseg <= 256 ? 1 : 0; }
  // GEMM job descriptors of the matrix-core stages (see k_gemm_stream).
  GemmJob near_job(const CT* x, CT* y, int R, int rt) const {
    const int nf = 2 * n_;
    GemmJob j{};
    j.A = A_near_.template as<float>();
    j.Ah = A_near_h_.template as<unsigned short>();
    j.Al = A_near_l_.template as<unsigned short>();
    j.B = reinterpret_cast<const float*>(x);
    j.bcol = near_nbr_.template as<int>();
    j.C = reinterpret_cast<float*>(y);
    j.ccol = iota_.template as<int>();
    j.sB = j.sC = (size_t)P_ * nf;
    j.M = nf;
    j.ncols = P_;
    j.nseg = 9;
    j.kseg = nf;
    j.lda = 9 * nf;
    j.ldb = j.ldc = nf;
    j.acc = 0;
    j.tiles_m = (nf + 16 * rt - 1) / (16 * rt);
    j.tiles = j.tiles_m * ((P_ + 15) / 16);
    (void)R;
    return j;
  }
  // U0 = radiation matrix of each particle's class times x (eq. kspace_Rap)
  GemmJob project_job(const CT* x, int rt) const {
    const int nf = 2 * n_;
    GemmJob j{};
    j.A = A_proj_.template as<float>();
    j.Ah = A_proj_h_.template as<unsigned short>();
    j.Al = A_proj_l_.template as<unsigned short>();
    j.a_off = a_off_proj_.template as<int>();
    j.B = reinterpret_cast<const float*>(x);
    j.bcol = gcol_part_.template as<int>();
    j.C = reinterpret_cast<float*>(pS_[0]);
    j.ccol = gcol_box_.template as<int>();
    j.sB = (size_t)P_ * nf;
    j.sC = (size_t)lv_[0].nx * lv_[0].ny * 2 * M2_;
    j.M = 2 * M2_;
    j.ncols = ncols_pad_;
    j.nseg = 1;
    j.kseg = nf;
    j.lda = nf;
    j.ldb = nf;
    j.ldc = 2 * M2_;
    j.acc = 0;
    j.tiles_m = (j.M + 16 * rt - 1) / (16 * rt);
    j.tiles = j.tiles_m * (ncols_pad_ / 16);
    j.wtile = short_k(j);
    return j;
  }
  // y += receiving matrix of each particle's class times G0 (eqs. Tmn_fmm, Kmn_fmm)
  GemmJob receive_job(CT* y, int rt) const {
    const int nf = 2 * n_;
    GemmJob j{};
    j.A = A_recv_.template as<float>();
    j.Ah = A_recv_h_.template as<unsigned short>();
    j.Al = A_recv_l_.template as<unsigned short>();
    j.a_off = a_off_recv_.template as<int>();
    j.B = reinterpret_cast<const float*>(pG_[0]);
    j.bcol = gcol_box_.template as<int>();
    j.C = reinterpret_cast<float*>(y);
    j.ccol = gcol_part_.template as<int>();
    j.sB = (size_t)lv_[0].nx * lv_[0].ny * 2 * M2_;
    j.sC = (size_t)P_ * nf;
    j.M = nf;
    j.ncols = ncols_pad_;
    j.nseg = 1;
    j.kseg = 2 * M2_;
    j.lda = 2 * M2_;
    j.ldb = 2 * M2_;
    j.ldc = nf;
    j.acc = 1;
    j.tiles_m = (j.M + 16 * rt - 1) / (16 * rt);
    j.tiles = j.tiles_m * (ncols_pad_ / 16);
    j.xcd = 1;  // the row tiles of one column tile read the same G0 columns
    return j;
  }
  // All translation levels, in two launches: LDS tiles on grids of at least
  // 8 x 8 boxes, and on all grids for batches of 4 or more RHS (for one RHS,
  // smaller grids waste most of a tile's halo and their gathered lists are
  // shorter), gathered lists on the others; largest level first so the small
  // ones fill the tail.  The 16-byte tile staging needs an even sample count
  // (np = 2L always is).
  void launch_translations(int R, hipStream_t st, double cb) {
    if constexpr (std::is_same<T, float>::value) {
      // FP32: every level in one launch of the register-tiled kernel (no LDS)
      if (tr_force_ < 0 || tr_force_ >= 4) {
        TrLevels<float> reg{};
        double bytes = 0, flops = 0;
        for (int l = 0; l < ntl_; ++l) {
          const Lvl& L = lv_[l];
          TrLevel<float>& V = reg.lv[reg.n++];
          V = TrLevel<float>{pS_[l], pG_[l],     L.TL.template as<CT>(), nullptr, nullptr, nullptr, L.nx,
                             L.ny,   L.K,    reg.total,                  L.TLp.template as<CP<float>>()};
          reg.total += ((L.nx + kTrRegTile - 1) / kTrRegTile) * ((L.ny + kTrRegTile - 1) / kTrRegTile) *
                       ((L.K + 63) / 64) * R;
          bytes += cb * (4.0 * R * L.nx * L.ny * L.K + 40.0 * L.K);
          flops += 16.0 * R * (double)pairs_[l] * L.K;
        }
        auto pr = begin("translate", bytes, flops);
        // mode 4 (the default): no column tests in interior tiles; modes 5-8:
        // column tests, source rows of interior tiles loaded 0, 1, 3 or 2 rows
        // ahead of the row being summed
        const dim3 g(xcd_grid(reg.total)), b(64);
        if (tr_force_ == 5) launch(pr, k_translate_reg<0, true>, g, b, 0u, st, reg, R);
        else if (tr_force_ == 6) launch(pr, k_translate_reg<1, true>, g, b, 0u, st, reg, R);
        else if (tr_force_ == 7) launch(pr, k_translate_reg<3, true>, g, b, 0u, st, reg, R);
        else if (tr_force_ == 8) launch(pr, k_translate_reg<2, true>, g, b, 0u, st, reg, R);
        else launch(pr, k_translate_reg<2, false>, g, b, 0u, st, reg, R);
        return;
      }
    }
    TrLevels<T> tiled{}, gath{};
    const int rpb = std::min(R, tr_rpb_);  // RHS per tiled block
    double tb = 0, tf = 0, gbytes = 0, gf = 0;
    int trm_all = 0;
    for (int l = 0; l < ntl_; ++l) {
      const Lvl& L = lv_[l];
      // LDS tiles on grids of at least 8 x 8 boxes, and on every grid once
      // several RHS share the launch (the gathered lists re-read each source
      // sample 27 times from L2)
      const int trm = L.K % 2 != 0 ? 0 : tr_force_ >= 0 ? tr_force_ : ((L.nx >= 8 && L.ny >= 8) || R >= 4 ? 1 : 0);
      TrLevels<T>& D = trm ? tiled : gath;
      TrLevel<T>& V = D.lv[D.n++];
      V = TrLevel<T>{pS_[l], pG_[l], L.TL.template as<CT>(),
                     L.il_cnt.template as<int>(), L.il_src.template as<int>(), L.il_off.template as<int>(),
                     L.nx, L.ny, L.K, D.total};
      const double bytes = cb * (4.0 * R * L.nx * L.ny * L.K + 40.0 * L.K), flops = 16.0 * R * (double)pairs_[l] * L.K;
      if (trm) {
        trm_all = trm;
        const int TX = trm == 1 ? 4 : 8, TY = trm == 3 ? 8 : 4, NS = TrNS<T>::v;
        D.total += ((L.nx + TX - 1) / TX) * ((L.ny + TY - 1) / TY) * ((L.K + NS - 1) / NS) * ((R + rpb - 1) / rpb);
        tb += bytes;
        tf += flops;
      } else {
        D.total += L.nx * L.ny * R * ((L.K + kBlock - 1) / kBlock);
        gbytes += bytes;
        gf += flops;
      }
    }
    const dim3 blk(kBlock);
    if (tiled.n) {
      auto pr = begin("translate_tiled", tb, tf);
      const dim3 g(xcd_grid(tiled.total));
      if (trm_all == 1)
        launch(pr, k_translate_tiled<T, 4, 4>, g, blk, 0u, st, tiled, R, rpb);
      else if (trm_all == 2)
        launch(pr, k_translate_tiled<T, 8, 4>, g, blk, 0u, st, tiled, R, rpb);
      else
        launch(pr, k_translate_tiled<T, 8, 8>, g, blk, 0u, st, tiled, R, rpb);
    }
    if (gath.n) {
      auto pr = begin("translate", gbytes, gf);
      launch(pr, k_translate<T>, dim3(xcd_grid(gath.total)), blk, 0u, st, gath, R);
    }
  }
  // The FP32 job with its R right-hand sides folded into the columns and
  // ct column tiles per block (ct divides R, so that a block stays within
  // one group of columns sharing A)
  static GemmJob fold_job(GemmJob j, int R, int ct) {
    if (!j.A) return j;
    j.fold = R;
    j.ncols *= R;
    j.tiles = j.tiles_m * ((j.ncols + 16 * ct - 1) / (16 * ct));
    return j;
  }
  // rt: 16-row MFMA tiles per block (1, 2 or 4; the jobs' tiles_m must use
  // it).  FP32: the RHS are folded into the columns and a block takes up to
  // 4 column tiles, so one read of a block's A rows serves 64 columns;
  // BF16-split: one grid layer per RHS.
  template <int Tag>
  void launch_gemm(Pending& pr, int rt, const GemmJob& j0u, const GemmJob& j1u, int R, hipStream_t st) {
    if (bf16_) {
      const int nt = gemm_blocks(j0u, 4) + gemm_blocks(j1u, 4);
      const dim3 grid(j0u.xcd ? xcd_grid(nt) : nt, 1, R);
      if (rt == 1)
        launch(pr, k_gemm_bf16x3<1, Tag>, grid, dim3(kBlock), 0u, st, j0u, j1u);
      else if (rt == 2)
        launch(pr, k_gemm_bf16x3<2, Tag>, grid, dim3(kBlock), 0u, st, j0u, j1u);
      else
        launch(pr, k_gemm_bf16x3<4, Tag>, grid, dim3(kBlock), 0u, st, j0u, j1u);
      return;
    }
    // the LDS-staged kernel where both jobs take the same mode and blocks of
    // W * CT column tiles stay inside one column group (W * CT divides R)
    const int md0 = lds_mode(j0u), md1 = j1u.A ? lds_mode(j1u) : md0;
    if (gemm_lds_ && md0 >= 0 && md0 == md1) {
      int W = 0, C = 0;
      lds_config(md0, R, W, C);
      if (W) {
        GemmJob a = j0u, b = j1u;
        a.fold = R;
        if (b.A) b.fold = R;
        const dim3 grid(8 * ((lds_blocks(a, W, C) + 7) / 8 + (lds_blocks(b, W, C) + 7) / 8)), blk(64 * W);
        if (md0 == 0 && C == 2) launch(pr, k_gemm_lds<0, 8, 2, Tag>, grid, blk, 0u, st, a, b);
        else if (md0 == 0 && W == 8) launch(pr, k_gemm_lds<0, 8, 1, Tag>, grid, blk, 0u, st, a, b);
        else if (md0 == 0) launch(pr, k_gemm_lds<0, 4, 1, Tag>, grid, blk, 0u, st, a, b);
        else if (W == 8) launch(pr, k_gemm_lds<1, 8, 1, Tag>, grid, blk, 0u, st, a, b);
        else launch(pr, k_gemm_lds<1, 4, 1, Tag>, grid, blk, 0u, st, a, b);
        return;
      }
    }
    const int ct = R % 4 == 0 ? 4 : R % 2 == 0 ? 2 : 1;
    const GemmJob j0 = fold_job(j0u, R, ct), j1 = fold_job(j1u, R, ct);
    const int nt = gemm_blocks(j0, kGemmW) + gemm_blocks(j1, kGemmW);
    const dim3 grid(j0.xcd ? xcd_grid(nt) : nt, 1, 1);
    const dim3 blk(64 * kGemmW);
    if (ct == 4) {
      if (rt == 1) launch(pr, k_gemm_stream<1, 4, Tag, kGemmW>, grid, blk, 0u, st, j0, j1);
      else if (rt == 2) launch(pr, k_gemm_stream<2, 4, Tag, kGemmW>, grid, blk, 0u, st, j0, j1);
      else launch(pr, k_gemm_stream<4, 4, Tag, kGemmW>, grid, blk, 0u, st, j0, j1);
    } else if (ct == 2) {
      if (rt == 1) launch(pr, k_gemm_stream<1, 2, Tag, kGemmW>, grid, blk, 0u, st, j0, j1);
      else if (rt == 2) launch(pr, k_gemm_stream<2, 2, Tag, kGemmW>, grid, blk, 0u, st, j0, j1);
      else launch(pr, k_gemm_stream<4, 2, Tag, kGemmW>, grid, blk, 0u, st, j0, j1);
    } else {
      if (rt == 1) launch(pr, k_gemm_stream<1, 1, Tag, kGemmW>, grid, blk, 0u, st, j0, j1);
      else if (rt == 2) launch(pr, k_gemm_stream<2, 1, Tag, kGemmW>, grid, blk, 0u, st, j0, j1);
      else launch(pr, k_gemm_stream<4, 1, Tag, kGemmW>, grid, blk, 0u, st, j0, j1);
    }
  }

  // the disaggregation kernel of a stencil order, tap count and strip width
  template <int ORD, int NT>
  void launch_dis_nt(Pending& pr, bool two, dim3 g, uint32_t sh, hipStream_t st, const InterpArgs<T>& A) {
    if (two)
      launch(pr, k_dis_stream<T, ORD, NT, 16>, g, dim3(64), sh, st, A);
    else
      launch(pr, k_dis_stream<T, ORD, NT, 32>, g, dim3(64), sh, st, A);
  }
  void launch_dis(Pending& pr, int order, int ntap, bool two, dim3 g, uint32_t sh, hipStream_t st,
                  const InterpArgs<T>& A) {
    if (order == 6) {
      if (ntap == 8) launch_dis_nt<6, 8>(pr, two, g, sh, st, A);
      else if (ntap == 10) launch_dis_nt<6, 10>(pr, two, g, sh, st, A);
      else if (ntap == 12) launch_dis_nt<6, 12>(pr, two, g, sh, st, A);
      else launch_dis_nt<6, 16>(pr, two, g, sh, st, A);
    } else {
      if (ntap == 8) launch_dis_nt<4, 8>(pr, two, g, sh, st, A);
      else if (ntap == 12) launch_dis_nt<4, 12>(pr, two, g, sh, st, A);
      else launch_dis_nt<4, 16>(pr, two, g, sh, st, A);
    }
  }

  // Arguments of the streamed interpolation between level l - 1 (child) and
  // l (parent) for R right-hand sides (chunk tables of batch bucket bk).
  InterpArgs<T> interp_args(int l, int R, int bk, bool agg) const {
    const Lvl &C = lv_[l - 1], &Pp = lv_[l];
    const Itp& I = it_[l];
    InterpArgs<T> A{};
    A.src = agg ? pS_[l - 1] : pG_[l];
    A.dst = agg ? pS_[l] : pG_[l - 1];
    A.E = I.E.template as<CP<T>>();
    A.chunk = (agg ? I.chunk_a.template as<int>() : I.chunk_d.template as<int>()) + (agg ? I.a_coff[bk] : I.d_coff[bk]);
    A.chunk_p = agg ? nullptr : I.chunkp_d.template as<int>() + 2 * (I.d_coff[bk] - bk);
    A.s0 = I.s0.template as<int>();
    A.thw = agg ? I.thw_a.template as<T>() : I.thw_d.template as<T>();
    A.vrow = I.vrow.template as<int>();
    A.vflip = I.vflip.template as<int>();
    A.colb = agg ? I.colb_a.template as<int>() : I.colb_d.template as<int>();
    A.colw = agg ? I.colw_a.template as<T>() : I.colw_d.template as<T>();
    A.wlo = agg ? I.wlo_a.template as<int>() : I.wlo_d.template as<int>();
    A.nxc = C.nx;
    A.nyc = C.ny;
    A.ntc = C.nt;
    A.npc = C.np;
    A.nxp = Pp.nx;
    A.nyp = Pp.ny;
    A.ntp = Pp.nt;
    A.npp = Pp.np;
    A.R = R;
    A.nst = agg ? I.a_nst : I.d_nst;
    A.nch = agg ? I.a_nch[bk] : I.d_nch[bk];
    A.wlen = agg ? I.a_wlen : I.d_wlen;
    A.ntap = agg ? I.order : I.d_ntap;
    return A;
  }

  // One product y = Z x: near-field apply and leaf projection (one launch on
  // the matrix cores), aggregation up the tree, then from the top level down
  // translation and disaggregation, and receive.
  int enqueue(const void* xv, void* yv, int R, int parts, hipStream_t st, std::string& err) {
    const CT* x = reinterpret_cast<const CT*>(xv);
    CT* y = reinterpret_cast<CT*>(yv);
    const dim3 blk(kBlock);
    const double cb = sizeof(CT);
    const bool near = parts & 1, far = (parts & 2) && ntl_ > 0;
    const double near_bytes = cb * ((double)2 * R * P_ * n_ + (double)nslots_ * n_ * n_);
    const double near_flops = 8.0 * R * nnear_ * (double)n_ * n_;
    const double proj_bytes = cb * ((double)R * P_ * n_ + (double)R * P_ * M2_ + (double)nc_ * n_ * M2_);
    const double proj_flops = 8.0 * R * P_ * (double)n_ * M2_;
    // leaf-level pattern buffers (only when there is a far part)
    const Lvl* L0 = far ? &lv_[0] : nullptr;
    const int nb0 = far ? L0->nx * L0->ny : 0;
    const GemmJob none{};
    const bool near_mfma = mfma_ && near_uniform_, near_grouped = mfma_ && !near_uniform_;
    auto near_sum = [&]() {
      const int nf = 2 * n_;
      auto pr = begin("near_sum", 4.0 * R * (9.0 + 1.0) * P_ * nf, 0.0);
      launch(pr, k_near_sum, dim3(std::min(grid1d((size_t)P_ * nf / 4), 2048), R), blk, 0, st, P_, nf,
             (const float*)pNear_, (const int*)ng_has_.template as<int>(),
             reinterpret_cast<float*>(y));
    };
    if (near && far && (near_mfma || near_grouped)) {
      auto pr = begin("near+project", near_bytes + proj_bytes, near_flops + proj_flops);
      launch_gemm<0>(pr, rt_np_, near_grouped ? near_group_job(x, rt_np_) : near_job(x, y, R, rt_np_),
                     project_job(x, rt_np_), R, st);
    } else {
      if (near) {
        auto pr = begin("near", near_bytes, near_flops);
        if (near_mfma || near_grouped) {
          launch_gemm<1>(pr, rt_np_, near_grouped ? near_group_job(x, rt_np_) : near_job(x, y, R, rt_np_), none, R,
                         st);
          if (near_grouped) near_sum();
        } else
          launch_near(pr, x, y, R, near_mats_.template as<CT>(), near_nbr_.template as<int>(),
                      near_slot_.template as<int>(), near_tile_slot_.template as<int>(), 9, st);
      } else {
        const size_t cnt = (size_t)R * P_ * n_;
        hipLaunchKernelGGL(k_fill_zero<T>, dim3(grid1d(cnt)), blk, 0, st, y, cnt);
      }
      if (far) {
        auto pr = begin("project", proj_bytes, proj_flops);
        if (mfma_) {
          launch_gemm<2>(pr, rt_np_, project_job(x, rt_np_), none, R, st);
        } else {
          dim3 grid(ntiles_, (M2_ + kProjBlock - 1) / kProjBlock, R);
          size_t sh = (size_t)kTP * n_ * sizeof(CT);
          launch(pr, k_project<T, kTP>, grid, dim3(kProjBlock), sh, st, n_, P_, M2_, nb0, x,
                             pS_[0], Rm_.template as<CT>(), rm_off_.template as<int>(),
                             order_.template as<int>(), tile_start_.template as<int>(),
                             tile_count_.template as<int>(), tile_class_.template as<int>(),
                             box_of_.template as<int>());
        }
      }
    }
    if (far) {
      const int bk = chunk_bucket(R);
      for (int l = 1; l < ntl_; ++l) {
        const Lvl &C = lv_[l - 1], &Pp = lv_[l];
        const Itp& I = it_[l];
        InterpArgs<T> A = interp_args(l, R, bk, true);
        const int items = R * Pp.nx * Pp.ny * (I.a_sw == kIStrip ? 2 : 1) * I.a_nst * I.a_nch[bk];
        auto pr = begin("aggregate_l" + std::to_string(l),
                        cb * 2.0 * R * ((double)C.nx * C.ny * C.K + (double)Pp.nx * Pp.ny * Pp.K),
                        2.0 * R * (double)Pp.nx * Pp.ny * 2 * 4 *
                            (4.0 * (double)C.nt * Pp.np * I.order + 4.0 * Pp.K * I.order) + 16.0 * R * Pp.nx * Pp.ny * 2 * Pp.K);
        const uint32_t sh = (uint32_t)(2 * 64 * (I.a_sw == kIStrip ? kIStage / 2 : 3 * kIStage / 4) * sizeof(CT));
        const dim3 g(xcd_grid(items)), b64(64);
        const bool two = I.a_sw != kIStrip;
        if (I.order == 6 && I.a_ends <= 2)
          launch(pr, two ? k_agg_stream<T, 6, 16, 2> : k_agg_stream<T, 6, 32, 2>, g, b64, sh, st, A);
        else if (I.order == 6)
          launch(pr, two ? k_agg_stream<T, 6, 16, 3> : k_agg_stream<T, 6, 32, 3>, g, b64, sh, st, A);
        else
          launch(pr, two ? k_agg_stream<T, 4, 16, 3> : k_agg_stream<T, 4, 32, 3>, g, b64, sh, st, A);
      }
      launch_translations(R, st, cb);
      for (int l = ntl_ - 2; l >= 0; --l) {
        const Lvl &L = lv_[l], &Pp = lv_[l + 1];
        const Itp& I = it_[l + 1];
        InterpArgs<T> A = interp_args(l + 1, R, bk, false);
        const int items = R * Pp.nx * Pp.ny * (I.d_sw == kIStrip ? 2 : 1) * I.d_nst * I.d_nch[bk];
        // algorithmic bytes: the parent pattern read once (the child's
        // translated pattern is read and written once more by this kernel)
        auto pr = begin("disaggregate_l" + std::to_string(l), cb * 2.0 * R * (double)Pp.nx * Pp.ny * Pp.K,
                        2.0 * R * (double)Pp.nx * Pp.ny * 2 * 4 *
                            (4.0 * (double)Pp.nt * L.np * I.d_ntap + 4.0 * (double)Pp.nt * L.np * I.order));
        const uint32_t sh = (uint32_t)(2 * ((kIStrip / I.d_sw) * 8 * I.d_wlen + 6 * I.d_wlen + 64) * sizeof(CT));
        launch_dis(pr, I.order, I.d_ntap, I.d_sw != kIStrip, dim3(xcd_grid(items)), sh, st, A);
      }
      // with the receive on k_gemm_lds, the class-pair near sum goes into its store
      if (near && near_grouped) near_sum();
      {
        auto pr = begin("receive", cb * ((double)R * P_ * M2_ + 2.0 * R * P_ * n_ + (double)nc_ * n_ * M2_),
                        8.0 * R * P_ * (double)n_ * M2_);
        if (mfma_) {
          launch_gemm<3>(pr, rt_recv_, receive_job(y, rt_recv_), none, R, st);
        } else {
          dim3 grid(ntiles_, R);
          launch(pr, k_receive<T, kTP>, grid, blk, 0, st, n_, P_, M2_, nb0, y, pG_[0],
                             Qm_.template as<CT>(), qm_off_.template as<int>(), order_.template as<int>(),
                             tile_start_.template as<int>(), tile_count_.template as<int>(),
                             tile_class_.template as<int>(), box_of_.template as<int>());
        }
      }
    }
    HIP_TRY(hipGetLastError());
    return 0;
  }

  int fields(const void* xv, int R, int npts, const double* points, void* Ev, void* stream,
             std::string& err) override {
    if (ntl_ == 0) {
      err = "fields: the tree has no far level (the leaf patterns are not formed)";
      return -1;
    }
    const Lvl& L0 = lv_[0];
    if (L0.K > kBlock || fld_L_ > kFldMaxL) {
      err = "fields: the leaf sphere has more than " + std::to_string(kBlock) + " samples";
      return -1;
    }
    if (npts <= 0) return 0;
    if (int rc = ensure(R, err)) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const CT* x = reinterpret_cast<const CT*>(xv);
    // leaf patterns of x, as the projection stage of the product forms them
    Pending none;
    if (mfma_) {
      launch_gemm<2>(none, rt_np_, project_job(x, rt_np_), GemmJob{}, R, st);
    } else {
      dim3 grid(ntiles_, (M2_ + kProjBlock - 1) / kProjBlock, R);
      size_t sh = (size_t)kTP * n_ * sizeof(CT);
      launch(none, k_project<T, kTP>, grid, dim3(kProjBlock), sh, st, n_, P_, M2_, L0.nx * L0.ny, x,
             L0.S.template as<CT>(), Rm_.template as<CT>(), rm_off_.template as<int>(), order_.template as<int>(),
             tile_start_.template as<int>(), tile_count_.template as<int>(), tile_class_.template as<int>(),
             box_of_.template as<int>());
    }
    if ((size_t)npts * 3 * sizeof(double) > fld_pts_.bytes) HIP_TRY(fld_pts_.alloc((size_t)npts * 3 * sizeof(double)));
    HIP_TRY(hipMemcpyAsync(fld_pts_.p, points, (size_t)npts * 3 * sizeof(double), hipMemcpyHostToDevice, st));
    launch(none, k_fields<T>, dim3((npts + kFldPts - 1) / kFldPts, R), dim3(kBlock), 0u, st, P_, L0.K, fld_L_,
           fld_k_, fld_cen_.template as<double>(), box_of_.template as<int>(), L0.nx * L0.ny,
           (const CT*)L0.S.template as<CT>(), fld_tab_.template as<float>(), npts,
           (const double*)fld_pts_.template as<double>(), reinterpret_cast<CT*>(Ev));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));  // the host point array may be released on return
    return 0;
  }

  int precondition(const void* xv, void* yv, int R, void* stream, std::string& err) override {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    Pending none;
    if (mfma_ && !bf16_) {  // FP32: each class's inverse self block on the matrix cores, columns grouped by class
      launch_gemm<4>(none, rt_np_, precond_job(reinterpret_cast<const CT*>(xv), reinterpret_cast<CT*>(yv), rt_np_),
                     GemmJob{}, R, st);
    } else {
      launch_near(none, reinterpret_cast<const CT*>(xv), reinterpret_cast<CT*>(yv), R, zinv_.template as<CT>(),
                  self_nbr_.template as<int>(), self_slot_.template as<int>(), self_tile_slot_.template as<int>(), 1,
                  st);
    }
    HIP_TRY(hipGetLastError());
    return 0;
  }
  // y_p = Z_s(class p)^-1 x_p for every particle: the projection's column
  // grouping with the classes' inverse self blocks as A
  GemmJob precond_job(const CT* x, CT* y, int rt) const {
    const int nf = 2 * n_;
    GemmJob j{};
    j.A = A_zinv_.template as<float>();
    j.a_off = a_off_zinv_.template as<int>();
    j.B = reinterpret_cast<const float*>(x);
    j.bcol = gcol_part_.template as<int>();
    j.C = reinterpret_cast<float*>(y);
    j.ccol = gcol_part_.template as<int>();
    j.sB = j.sC = (size_t)P_ * nf;
    j.M = nf;
    j.ncols = ncols_pad_;
    j.nseg = 1;
    j.kseg = nf;
    j.lda = j.ldb = j.ldc = nf;
    j.acc = 0;
    j.tiles_m = (nf + 16 * rt - 1) / (16 * rt);
    j.tiles = j.tiles_m * (ncols_pad_ / 16);
    j.wtile = short_k(j);
    return j;
  }

  void launch_near(Pending& pr, const CT* x, CT* y, int R, const CT* mats, const int* nbr, const int* slot,
                   const int* tile_slot, int nsp, hipStream_t st) {
    dim3 grid((P_ + kTPN - 1) / kTPN, R);
    const size_t xs_bytes = (size_t)kTPN * n_ * sizeof(CT);
    const size_t m_bytes = (size_t)n_ * n_ * sizeof(CT);
    if (xs_bytes + m_bytes <= 64 * 1024)
      launch(pr, k_near<T, kTPN, true>, grid, dim3(kBlock), (uint32_t)(xs_bytes + m_bytes), st, n_, P_, nsp, x, y,
             mats, nbr, slot, tile_slot);
    else
      launch(pr, k_near<T, kTPN, false>, grid, dim3(kBlock), (uint32_t)xs_bytes, st, n_, P_, nsp, x, y, mats, nbr,
             slot, tile_slot);
  }

  int rhs(const std::vector<cd>& pat, const std::vector<V3>& khat, int R, void* b, void* stream,
          std::string& err) override {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const double k = 2.0 * kPi;
    std::vector<cd> phase((size_t)R * P_);
    for (int r = 0; r < R; ++r)
      for (int p = 0; p < P_; ++p) {
        const double a = -k * dot(khat[r], centers_[p]);
        phase[(size_t)r * P_ + p] = cd(std::cos(a), std::sin(a));
      }
    DevMem dpat, dph;
    if (int rc = put_c(dpat, pat, err)) return rc;
    if (int rc = put_c(dph, phase, err)) return rc;
    const size_t cnt = (size_t)R * P_ * n_;
    hipLaunchKernelGGL(k_rhs<T>, dim3(grid1d(cnt)), dim3(kBlock), 0, st, n_, P_, R, dpat.template as<CT>(),
                       class_of_.template as<int>(), dph.template as<CT>(), reinterpret_cast<CT*>(b));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));  // dpat/dph are released on return
    return 0;
  }

  int gmres(const void* bv, void* xv, int R, double rtol, int max_iter, int m, bool use_x0, bool always_reorth,
            bool fp32_basis, std::vector<GmresResult>& res, void* stream, std::string& err) override;
  template <typename VB>
  int gmres_t(const void* bv, void* xv, int R, double rtol, int max_iter, int m, bool use_x0, bool always_reorth,
              std::vector<GmresResult>& res, void* stream, std::string& err);

  void profile(bool enable) override {
    prof_on_ = enable;
    for (auto& r : rec_) pool_.push_back(r.a), pool_.push_back(r.b);
    rec_.clear();
    table_.clear();
    stage_index_.clear();
  }

  int profile_read(std::vector<StageTime>& out, std::string& err) override {
    for (auto& r : rec_) {
      HIP_TRY(hipEventSynchronize(r.b));
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
      table_[r.stage].total_ms += ms;
      table_[r.stage].launches += 1;
      pool_.push_back(r.a);
      pool_.push_back(r.b);
    }
    rec_.clear();
    out = table_;
    return 0;
  }

  long long device_bytes() const override {
    long long s = 0;
    for (auto& L : lv_) s += L.TL.bytes + L.TLp.bytes + L.S.bytes + L.G.bytes;
    for (auto& I : it_)
      s += I.s0.bytes + I.vrow.bytes + I.vflip.bytes + I.thw_a.bytes + I.thw_d.bytes + I.colb_a.bytes +
           I.colw_a.bytes + I.colb_d.bytes + I.colw_d.bytes + I.wlo_a.bytes + I.wlo_d.bytes + I.E.bytes +
           I.chunk_a.bytes + I.chunk_d.bytes + I.chunkp_d.bytes;
    s += Rm_.bytes + Qm_.bytes + near_mats_.bytes + zinv_.bytes + box_of_.bytes + order_.bytes + near_nbr_.bytes +
         near_slot_.bytes;
    return s;
  }

 private:
  static constexpr int kTP = sizeof(T) == 4 ? 16 : 8;
  static constexpr int kTPN = 16;
  int rt_np_ = 4, rt_recv_ = 4;  // MFMA GEMM row tiles (of 16) per block: near+projection, receive
  static constexpr size_t kLdsBudget = 48 * 1024;  // preferred tile size (occupancy)
  static constexpr size_t kLdsMax = 64 * 1024;     // hard limit per block
  static constexpr size_t kStreamItems = 4096;  // waves per streamed interpolation launch (target)

  template <typename U>
  static int put_raw(DevMem& d, const U* h, size_t count, std::string& err) {
    HIP_TRY(d.alloc(count * sizeof(U)));
    if (count) HIP_TRY(hipMemcpy(d.p, h, count * sizeof(U), hipMemcpyHostToDevice));
    return 0;
  }
  static int put_i(DevMem& d, const std::vector<int>& v, std::string& err) { return put_raw(d, v.data(), v.size(), err); }
  static int put_u8(DevMem& d, const std::vector<uint8_t>& v, std::string& err) {
    std::vector<int> w(v.begin(), v.end());
    return put_raw(d, w.data(), w.size(), err);
  }
  static int put_r(DevMem& d, const std::vector<double>& v, std::string& err) {
    std::vector<T> w(v.begin(), v.end());
    return put_raw(d, w.data(), w.size(), err);
  }
  static int put_c(DevMem& d, const std::vector<cd>& v, std::string& err) {
    std::vector<CT> w(v.size());
    for (size_t i = 0; i < v.size(); ++i) w[i] = {(T)v[i].real(), (T)v[i].imag()};
    return put_raw(d, w.data(), w.size(), err);
  }

  bool prof_on_ = false;
  std::vector<StageTime> table_;
  std::map<std::string, int> stage_index_;
  int cur_stage_ = -1;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool_;
  std::vector<Rec> rec_;

  void register_stage(const std::string& name, double bytes, double flops) {
    auto it = stage_index_.find(name);
    if (it == stage_index_.end()) {
      StageTime t;
      t.name = name;
      t.bytes = bytes;
      t.flops = flops;
      table_.push_back(t);
      it = stage_index_.emplace(name, (int)table_.size() - 1).first;
    }
    cur_stage_ = it->second;
  }

  struct GraphEntry {
    const void* x = nullptr;
    void* y = nullptr;
    int R = 0, parts = 0;
    hipGraphExec_t exec = nullptr;
    unsigned long long used = 0;
  };
  static constexpr size_t kMaxGraphs = 32;
  std::vector<GraphEntry> graphs_;
  hipStream_t cap_stream_ = nullptr;
  unsigned long long use_clock_ = 0;
  bool use_graphs_ = std::getenv("MLFMA_NO_GRAPH") == nullptr;
  // GMRES launches its kernels directly unless MLFMA_GMRES_GRAPHS is set:
  // then the product and the Arnoldi step are replayed graphs.  Each graph
  // boundary costs about 8 us of idle GPU on ROCm 7 (the next dispatch
  // waits for the graph's completion signal), more than the host's launch
  // time it saves.
  bool gmres_graphs_ = std::getenv("MLFMA_GMRES_GRAPHS") != nullptr;
  bool gmres_progress_ = std::getenv("MLFMA_GMRES_PROGRESS") != nullptr;
  // FP32 GEMMs through the LDS-staged kernel where it applies (MLFMA_GEMM=stream: always k_gemm_stream)
  bool gemm_lds_ = [] {
    const char* e = std::getenv("MLFMA_GEMM");
    return !(e && std::string(e) == "stream");
  }();

  static void destroy_entry(GraphEntry& e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    e.exec = nullptr;
  }
  void clear_graphs() {
    for (auto& e : graphs_) destroy_entry(e);
    graphs_.clear();
  }

 public:
  ~EngineT() override {
    (void)hipDeviceSynchronize();
    clear_graphs();
    for (auto e : pool_) (void)hipEventDestroy(e);
    for (auto& r : rec_) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
    if (col_ev_) (void)hipEventDestroy(col_ev_);
  }

 private:
  // Profiling: each stage is one kernel launch; while profiling it goes
  // through hipExtLaunchKernel with a start and a stop event, which time the
  // dispatch itself on the launch stream (direct launches only; the product
  // is not graph-captured while profiling).
  Pending begin(const std::string& name, double bytes, double flops) {
    if (!prof_on_) return {};
    register_stage(name, bytes, flops);
    return {cur_stage_, take_event(), take_event()};
  }
  template <typename F, typename... Args>
  void launch(Pending& p, F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t st, Args... args) {
    if (p.a) {
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, p.a, p.b, 0, args...);
      rec_.push_back({p.stage, p.a, p.b});
      if (table_[p.stage].kernel.empty()) table_[p.stage].kernel = kernel_symbol(reinterpret_cast<const void*>(kernel), st);
      p = Pending{};
    } else {
      hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
    }
  }
  hipEvent_t take_event() {
    if (!pool_.empty()) {
      hipEvent_t e = pool_.back();
      pool_.pop_back();
      return e;
    }
    hipEvent_t e{};
    (void)hipEventCreate(&e);
    return e;
  }

  int N_ = 0, n_ = 0, P_ = 0, nc_ = 0, ntl_ = 0, nx0_ = 0, ny0_ = 0, ntiles_ = 0, tp_ = 0, M2_ = 0, R_alloc_ = 0;
  CT* pS_[kMaxTrLv] = {};  // pattern buffers in use (see bind_context_buffers)
  CT* pG_[kMaxTrLv] = {};
  float* pNear_ = nullptr;
  std::vector<Lvl> lv_;
  std::vector<Itp> it_;
  const Tree* tree_ = nullptr;
  DevMem box_of_, class_of_, order_, tile_start_, tile_count_, tile_class_;
  DevMem fld_cen_, fld_tab_, fld_pts_;  // field evaluation: centres, leaf sample table, points
  double fld_k_ = 0;
  int fld_L_ = 0;
  DevMem Rm_, Qm_, rm_off_, qm_off_;
  DevMem near_mats_, near_nbr_, near_slot_, zinv_, self_nbr_, self_slot_, near_tile_slot_, self_tile_slot_;
  bool mfma_ = false, near_uniform_ = false;
  int tr_rpb_ = 1;  // RHS per block of the tiled translation (16 measured slower on the full-scale lens)
  // translation kernel forced on every level: 0 = gathered lists, 1/2/3 = LDS
  // tiles of 4x4 / 8x4 / 8x8 boxes, 4 = register tiles (FP32), 5-8 = register
  // tiles with column tests (FP32, rows loaded 0, 1, 3, 2 ahead); -1 = the
  // default (register tiles in FP32; in FP64 LDS tiles of 4x4 on grids of at
  // least 8 x 8 boxes or with 4 or more RHS, gathered lists otherwise)
  int tr_force_ = [] {
    const char* e = std::getenv("MLFMA_TRANSLATE");
    const int m = e ? std::atoi(e) : -1;
    return m >= 0 && m <= (std::is_same<T, float>::value ? 8 : 3) ? m : -1;
  }();
  DevMem A_proj_, A_recv_, A_near_, iota_;
  DevMem A_proj_h_, A_proj_l_, A_recv_h_, A_recv_l_, A_near_h_, A_near_l_;  // BF16-split copies
  bool bf16_ = false;  // dense contractions as BF16-split matrix-core products
  DevMem gcol_part_, gcol_box_, a_off_proj_, a_off_recv_;  // class-grouped GEMM columns
  DevMem A_zinv_, a_off_zinv_;  // the preconditioner's inverse self blocks for the matrix cores
  DevMem ng_bcol_, ng_ccol_, ng_aoff_, ng_has_, near_part_;  // class-pair near GEMM
  int ngcols_ = 0;
  int ncols_pad_ = 0;
  std::vector<V3> centers_;
  int nslots_ = 0;
  long long nnear_ = 0;
  std::vector<long long> pairs_;
  // GMRES workspace
  DevMem gV_, gw_, gx_, gb_, gtmp_, gtmpT_, gtmpT2_, gpart_, gh_, gh2_, gcol_, gn_, ggate_, gscale_, gstep_;
  HostMem hcol_, hy_;
  hipEvent_t col_ev_ = nullptr;
};

// Right-preconditioned restarted GMRES, Arnoldi in FP64 by classical
// Gram-Schmidt with selective (DGKS) or unconditional reorthogonalisation.
// Each RHS has its own Krylov space; all RHS advance in lock-step and
// converged ones are frozen (their Hessenberg columns are no longer updated,
// so their correction coefficients are zero).  Per iteration the host waits
// once, for the Hessenberg column; the next product is already queued.
template <typename T>
int EngineT<T>::gmres(const void* bv, void* xv, int R, double rtol, int max_iter, int m, bool use_x0,
                      bool always_reorth, bool fp32_basis, std::vector<GmresResult>& res, void* stream,
                      std::string& err) {
  if (fp32_basis) return gmres_t<float>(bv, xv, R, rtol, max_iter, m, use_x0, always_reorth, res, stream, err);
  return gmres_t<double>(bv, xv, R, rtol, max_iter, m, use_x0, always_reorth, res, stream, err);
}

// VB: precision the Krylov basis is stored in (all Arnoldi arithmetic is FP64)
template <typename T>
template <typename VB>
int EngineT<T>::gmres_t(const void* bv, void* xv, int R, double rtol, int max_iter, int m, bool use_x0,
                        bool always_reorth, std::vector<GmresResult>& res, void* stream, std::string& err) {
  using CV = C2<VB>;
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const size_t Nt = (size_t)P_ * n_;
  const size_t tot = (size_t)R * Nt;
  const size_t vstride = tot;  // V[i] is [R][Nt]
  const int ld = m + 2;        // per-RHS coefficient slots: m + 1 dots/norm + gate
  const int nblk_d = (int)std::min<size_t>(kDotMaxBlocks, (Nt + kBlock * kDotE - 1) / (kBlock * kDotE));
  const int nblk_s = (int)std::min<size_t>(1024, (Nt + kBlock - 1) / kBlock);
  HIP_TRY(gV_.alloc((size_t)(m + 1) * tot * sizeof(CV)));
  HIP_TRY(gw_.alloc(tot * sizeof(Z)));
  HIP_TRY(gx_.alloc(tot * sizeof(Z)));
  HIP_TRY(gb_.alloc(tot * sizeof(Z)));
  HIP_TRY(gtmp_.alloc(tot * sizeof(Z)));
  HIP_TRY(gtmpT_.alloc(tot * sizeof(CT)));
  HIP_TRY(gtmpT2_.alloc(tot * sizeof(CT)));
  HIP_TRY(gpart_.alloc((size_t)R * ld * std::max(nblk_d, nblk_s) * sizeof(Z)));
  HIP_TRY(gh_.alloc((size_t)R * ld * sizeof(Z)));
  HIP_TRY(gh2_.alloc((size_t)R * ld * sizeof(Z)));
  HIP_TRY(gcol_.alloc((size_t)R * ld * sizeof(Z)));
  HIP_TRY(gn_.alloc((size_t)2 * R * sizeof(Z)));
  HIP_TRY(ggate_.alloc((size_t)R * sizeof(int)));
  HIP_TRY(gstep_.alloc(sizeof(int)));
  HIP_TRY(gscale_.alloc((size_t)R * sizeof(double)));
  HIP_TRY(hcol_.alloc((size_t)R * ld * sizeof(Z)));
  HIP_TRY(hy_.alloc((size_t)R * ld * sizeof(Z)));
  if (!col_ev_) HIP_TRY(hipEventCreateWithFlags(&col_ev_, hipEventDisableTiming));
  CV* V = gV_.as<CV>();
  Z* w = gw_.as<Z>();
  Z* x = gx_.as<Z>();
  Z* b = gb_.as<Z>();
  Z* tmp = gtmp_.as<Z>();
  CT* tT = gtmpT_.as<CT>();
  CT* tT2 = gtmpT2_.as<CT>();
  Z* part = gpart_.as<Z>();
  Z* h1 = gh_.as<Z>();
  Z* h2 = gh2_.as<Z>();
  Z* col = gcol_.as<Z>();
  Z* n1 = gn_.as<Z>();
  Z* n2 = n1 + R;
  int* gate = ggate_.as<int>();
  double* scale = gscale_.as<double>();
  Z* hcol = hcol_.as<Z>();
  Z* hy = hy_.as<Z>();
  const dim3 blk(kBlock);
  const dim3 gv(grid1d(Nt) > 1024 ? 1024 : grid1d(Nt), R);
  // h[r][0..nv) = V_i^H w_r, and h[r][nv] = |w_r|^2 when want_norm
  int* jd_dev = gstep_.as<int>();
  // groups of basis vectors: enough blocks for kDotMinBlocks, each group a
  // multiple of the vectors one step loads.  With jd (graph replay) the
  // launch is shaped for the longest basis, m vectors, and the kernels read
  // the basis length from the device.
  const int gcap = (kDotMinBlocks + nblk_d - 1) / nblk_d;
  auto dots_on = [&](hipStream_t s, int nv, int want_norm, const Z* ww, Z* out, int ldo, const int* g,
                     const int* jd) {
    constexpr int VU = dot_vu<VB>();
    const int nl = jd ? m : nv;
    int gsz = dot_group(nl, VU, gcap), ng = nl > 0 ? (nl + gsz - 1) / gsz : 1;
    if (jd)  // every basis length up to m: the largest group and group count
      for (int n = 1; n <= m; ++n) {
        const int gn = dot_group(n, VU, gcap);
        gsz = std::max(gsz, gn);
        ng = std::max(ng, (n + gn - 1) / gn);
      }
    hipLaunchKernelGGL(k_dots<VB>, dim3(nblk_d, ng, R), blk, (uint32_t)((gsz + want_norm) * (kBlock / 64) * sizeof(Z)),
                       s, nv, want_norm, gsz, gcap, Nt, vstride, (const CV*)V, ww, part, ld, g, jd);
    hipLaunchKernelGGL(k_reduce, dim3(nl + want_norm, R), blk, 0, s, nblk_d, part, ld, out, ldo, g, jd, want_norm);
  };
  auto dots = [&](int nv, int want_norm, const Z* ww, Z* out, int ldo, const int* g) {
    dots_on(st, nv, want_norm, ww, out, ldo, g, nullptr);
  };
  // ww -= sum_i V_i c_i; nout[r] = |ww_r|^2
  auto subtract_on = [&](hipStream_t s, int nv, const Z* c, Z* ww, Z* nout, const int* g, const int* jd) {
    hipLaunchKernelGGL(k_subtract_norm<VB>, dim3(nblk_s, R), blk, 0, s, nv, Nt, vstride, (const CV*)V, c, ld, ww,
                       part, g, jd);
    hipLaunchKernelGGL(k_reduce, dim3(1, R), blk, 0, s, nblk_s, part, 1, nout, 1, g, nullptr, 0);
  };
  // Arnoldi step j on w = A v_j: two Gram-Schmidt passes, the second where
  // DGKS asks for it; the Hessenberg column to col (and to the host), v_{j+1}
  // = w / |w|, also written to tT for the next product when conv_next.  With
  // jd: j is read from the device, v_{j+1} always goes to tT, and *jd
  // advances, so that the same launches (one captured graph) serve every
  // step.
  auto arnoldi_step = [&](hipStream_t s, int j, const int* jd, bool conv_next) -> int {
    const int nv = j + 1;
    dots_on(s, nv, 1, w, h1, ld, nullptr, jd);
    subtract_on(s, nv, h1, w, n1, nullptr, jd);
    hipLaunchKernelGGL(k_dgks_gate, dim3((R + 63) / 64), dim3(64), 0, s, R, h1, ld, nv, n1, gate,
                       always_reorth ? 1 : 0, jd);
    dots_on(s, nv, 0, w, h2, ld, gate, jd);
    subtract_on(s, nv, h2, w, n2, gate, jd);
    hipLaunchKernelGGL(k_arnoldi_col, dim3(R), blk, 0, s, nv, ld, h1, n1, h2, n2, gate, col, scale, jd);
    hipLaunchKernelGGL((k_scale_real<VB, T>), gv, blk, 0, s, Nt, (const Z*)w, (const double*)scale,
                       jd ? V : V + (size_t)(j + 1) * vstride, (jd || conv_next) ? tT : (CT*)nullptr, vstride, jd);
    HIP_TRY(hipMemcpyAsync(hcol, col, (size_t)R * ld * sizeof(Z), hipMemcpyDeviceToHost, s));
    if (jd) hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, jd_dev, 1, 1);
    return 0;
  };
  // operator A z = Z (P^-1 z) -> result FP64 in `out`; z is a basis vector
  // (precond) or an FP64 iterate
  // (A_converted: z already converted into tT)
  auto apply_A_converted = [&](Z* out, bool precond) -> int {
    const CT* src = tT;
    if (precond) {
      if (int rc = precondition(tT, tT2, R, stream, err)) return rc;
      src = tT2;
    }
    CT* dst = precond ? tT : tT2;
    if (gmres_graphs_) {
      if (int rc = matvec(src, dst, R, 3, stream, err)) return rc;
    } else {
      const int old_alloc = R_alloc_;
      if (int rc = ensure(R, err)) return rc;
      if (R_alloc_ != old_alloc) clear_graphs();
      if (int rc = enqueue(src, dst, R, 3, st, err)) return rc;
    }
    hipLaunchKernelGGL(k_to_z<T>, dim3(grid1d(tot)), blk, 0, st, dst, out, tot);
    return 0;
  };
  auto apply_A_from = [&](auto* z, Z* out, bool precond) -> int {
    using S = typename std::remove_const<typename std::remove_pointer<decltype(z)>::type>::type;
    hipLaunchKernelGGL((k_convert<decltype(S{}.x), T>), dim3(grid1d(tot)), blk, 0, st, (const S*)z, tT, tot);
    return apply_A_converted(out, precond);
  };
  auto apply_A = [&](const Z* z, Z* out, bool precond) -> int { return apply_A_from(z, out, precond); };
  auto norms = [&](const Z* vec, std::vector<double>& out) -> int {
    dots(0, 1, vec, n1, 1, nullptr);
    HIP_TRY(hipMemcpyAsync(hcol, n1, (size_t)R * sizeof(Z), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    out.resize(R);
    for (int r = 0; r < R; ++r)  // NaN or Inf in the vector stays visible (max would drop a NaN)
      out[r] = std::isfinite(hcol[r].x) ? std::sqrt(std::max(0.0, hcol[r].x)) : std::nan("");
    return 0;
  };
  hipLaunchKernelGGL(k_to_z<T>, dim3(grid1d(tot)), blk, 0, st, reinterpret_cast<const CT*>(bv), b, tot);
  if (use_x0)
    hipLaunchKernelGGL(k_to_z<T>, dim3(grid1d(tot)), blk, 0, st, reinterpret_cast<const CT*>(xv), x, tot);
  else
    HIP_TRY(hipMemsetAsync(x, 0, tot * sizeof(Z), st));
  std::vector<double> bnorm, rnorm;
  if (int rc = norms(b, bnorm)) return rc;
  // NaN or Inf anywhere in b (or in the guess) makes its squared norm
  // non-finite: rejected before the first product
  for (int r = 0; r < R; ++r)
    if (!std::isfinite(bnorm[r])) {
      err = "gmres: right-hand side " + std::to_string(r) + " holds NaN or Inf";
      return -5;
    }
  if (use_x0) {
    std::vector<double> xnorm;
    if (int rc = norms(x, xnorm)) return rc;
    for (int r = 0; r < R; ++r)
      if (!std::isfinite(xnorm[r])) {
        err = "gmres: initial guess " + std::to_string(r) + " holds NaN or Inf";
        return -5;
      }
  }
  res.assign(R, GmresResult{});
  // residual r = b - Z x
  auto residual = [&](Z* out) -> int {
    if (int rc = apply_A(x, tmp, false)) return rc;
    hipLaunchKernelGGL(k_sub, dim3(grid1d(tot)), blk, 0, st, tot, b, tmp, out);
    return 0;
  };
  if (int rc = residual(w)) return rc;
  if (int rc = norms(w, rnorm)) return rc;
  if (use_x0) {
    // scale each guess by the complex factor a = (A x0)^H b / |A x0|^2 that
    // minimises |b - a A x0|: never worse than a zero start (a = 0), which is
    // what a guess uncorrelated with the solution falls back to
    hipLaunchKernelGGL(k_guess_dots, dim3(nblk_d, R), blk, 0, st, Nt, (const Z*)tmp, (const Z*)b, part);
    hipLaunchKernelGGL(k_reduce, dim3(2, R), blk, 0, st, nblk_d, (const Z*)part, 2, n1, 2, nullptr, nullptr, 0);
    HIP_TRY(hipMemcpyAsync(hcol, n1, (size_t)2 * R * sizeof(Z), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int r = 0; r < R; ++r) {
      const double yy = hcol[2 * r + 1].x;
      cd a = yy > 0.0 ? cd(hcol[2 * r].x, hcol[2 * r].y) / yy : cd(0.0);
      if (!std::isfinite(a.real()) || !std::isfinite(a.imag())) a = 0.0;
      hy[r] = Z{a.real(), a.imag()};
    }
    HIP_TRY(hipMemcpyAsync(h1, hy, (size_t)R * sizeof(Z), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_guess_apply, gv, blk, 0, st, Nt, (const Z*)h1, x, (const Z*)tmp, (const Z*)b, w);
    if (int rc = norms(w, rnorm)) return rc;
  }
  std::vector<char> done(R, 0);
  std::vector<int> iters(R, 0), reorth(R, 0), cycles(R, 0);
  for (int r = 0; r < R; ++r) {
    if (bnorm[r] == 0.0 || rnorm[r] <= rtol * bnorm[r]) done[r] = 1;
  }
  // the Arnoldi step as one graph, captured on first use (not while
  // profiling, nor with graphs switched off)
  struct ExecGuard {
    hipGraphExec_t e = nullptr;
    ~ExecGuard() {
      if (e) (void)hipGraphExecDestroy(e);
    }
  } step_graph;
  const bool graph_steps = use_graphs_ && gmres_graphs_ && !prof_on_;
  auto capture_step = [&]() -> int {
    if (!cap_stream_) HIP_TRY(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal));
    const int rc = arnoldi_step(cap_stream_, 0, jd_dev, true);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(cap_stream_, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    HIP_TRY(ce);
    const hipError_t ie = hipGraphInstantiate(&step_graph.e, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIP_TRY(ie);
    return 0;
  };
  int total_it = 0;
  std::vector<std::vector<cd>> H(R), cs(R), sn(R), g(R);
  std::vector<double> s0(R);
  while (true) {
    bool all_done = true;
    for (int r = 0; r < R; ++r) all_done &= (bool)done[r];
    if (all_done || total_it >= max_iter) break;
    // V0 = r / |r| (zero for finished RHS so they stay frozen)
    for (int r = 0; r < R; ++r) {
      s0[r] = done[r] || rnorm[r] == 0.0 ? 0.0 : 1.0 / rnorm[r];
      H[r].assign((size_t)(m + 1) * m, 0.0);
      cs[r].assign(m, 0.0);
      sn[r].assign(m, 0.0);
      g[r].assign(m + 1, 0.0);
      g[r][0] = rnorm[r];
      if (!done[r]) cycles[r]++;
    }
    HIP_TRY(hipMemcpyAsync(scale, s0.data(), (size_t)R * sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL((k_scale_real<VB, T>), gv, blk, 0, st, Nt, (const Z*)w, (const double*)scale, V, tT, vstride,
                       (const int*)nullptr);
    int j = 0;
    std::vector<char> active(R);
    for (int r = 0; r < R; ++r) active[r] = !done[r];
    if (int rc = apply_A_converted(w, true)) return rc;  // v_0 is in tT
    if (graph_steps) {
      if (!step_graph.e)
        if (int rc = capture_step()) return rc;
      hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, st, jd_dev, 0, 0);
    }
    for (; j < m && total_it < max_iter; ++j) {
      ++total_it;
      const int nv = j + 1;
      const bool next = j + 1 < m && total_it < max_iter;
      if (graph_steps) {
        HIP_TRY(hipGraphLaunch(step_graph.e, st));
      } else if (int rc = arnoldi_step(st, j, nullptr, next)) {
        return rc;
      }
      HIP_TRY(hipEventRecord(col_ev_, st));
      // queue the next product (its input v_{j+1} is in tT) before the host
      // looks at the column
      if (next)
        if (int rc = apply_A_converted(w, true)) return rc;
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipEventSynchronize(col_ev_));
      bool any_active = false;
      for (int r = 0; r < R; ++r) {
        if (!active[r]) continue;
        iters[r]++;
        const Z* cr = hcol + (size_t)r * ld;
        reorth[r] += cr[nv + 1].x != 0.0;
        std::vector<cd>& Hr = H[r];
        for (int i = 0; i <= j; ++i) Hr[(size_t)i * m + j] = cd(cr[i].x, cr[i].y);
        const double wn = cr[nv].x;
        Hr[(size_t)(j + 1) * m + j] = wn;
        for (int i = 0; i < j; ++i) {  // previous rotations
          cd a = Hr[(size_t)i * m + j], bb = Hr[(size_t)(i + 1) * m + j];
          Hr[(size_t)i * m + j] = std::conj(cs[r][i]) * a + std::conj(sn[r][i]) * bb;
          Hr[(size_t)(i + 1) * m + j] = -sn[r][i] * a + cs[r][i] * bb;
        }
        cd a = Hr[(size_t)j * m + j], bb = Hr[(size_t)(j + 1) * m + j];
        double den = std::sqrt(std::norm(a) + std::norm(bb));
        if (den == 0.0) {
          cs[r][j] = 1.0;
          sn[r][j] = 0.0;
        } else {
          cs[r][j] = a / den;
          sn[r][j] = bb / den;
        }
        Hr[(size_t)j * m + j] = den;
        Hr[(size_t)(j + 1) * m + j] = 0.0;
        g[r][j + 1] = -sn[r][j] * g[r][j];
        g[r][j] = std::conj(cs[r][j]) * g[r][j];
        const double est = std::abs(g[r][j + 1]);
        if (!std::isfinite(est)) {
          err = "non-finite Arnoldi coefficient";
          return -5;  // non-finite
        }
        if (est <= rtol * bnorm[r] || wn == 0.0) active[r] = 0;
        any_active |= (bool)active[r];
      }
      if (!any_active) {
        ++j;
        break;
      }
    }
    // x += P^-1 V y with H y = g (upper triangular, per RHS, size j)
    for (size_t i = 0; i < (size_t)R * ld; ++i) hy[i] = Z{0, 0};
    for (int r = 0; r < R; ++r) {
      if (done[r]) continue;
      std::vector<cd> yy(j, 0.0);
      for (int i = j - 1; i >= 0; --i) {
        cd s = g[r][i];
        for (int k2 = i + 1; k2 < j; ++k2) s -= H[r][(size_t)i * m + k2] * yy[k2];
        cd d = H[r][(size_t)i * m + i];
        yy[i] = d == 0.0 ? 0.0 : s / d;
      }
      for (int i = 0; i < j; ++i) hy[(size_t)r * ld + i] = Z{yy[i].real(), yy[i].imag()};
    }
    HIP_TRY(hipMemcpyAsync(h1, hy, (size_t)R * ld * sizeof(Z), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_combine<VB>, gv, blk, 0, st, j, ld, Nt, vstride, (const CV*)V, (const Z*)h1, tmp, 0);
    // x += P^-1 tmp (through the context precision)
    hipLaunchKernelGGL(k_from_z<T>, dim3(grid1d(tot)), blk, 0, st, tmp, tT, tot);
    if (int rc = precondition(tT, tT2, R, stream, err)) return rc;
    hipLaunchKernelGGL(k_to_z<T>, dim3(grid1d(tot)), blk, 0, st, tT2, tmp, tot);
    hipLaunchKernelGGL(k_add, dim3(grid1d(tot)), blk, 0, st, tot, tmp, x);
    // true residual
    if (int rc = residual(w)) return rc;
    if (int rc = norms(w, rnorm)) return rc;
    for (int r = 0; r < R; ++r)
      if (!done[r] && rnorm[r] <= rtol * bnorm[r]) done[r] = 1;
    if (gmres_progress_) {  // one line per restart cycle (MLFMA_GMRES_PROGRESS)
      double worst = 0;
      int nd = 0;
      for (int r = 0; r < R; ++r) {
        worst = std::max(worst, bnorm[r] > 0 ? rnorm[r] / bnorm[r] : 0.0);
        nd += done[r] ? 1 : 0;
      }
      std::fprintf(stderr, "gmres: %d iterations, largest true rel. residual %.3e, %d of %d RHS converged\n",
                   total_it, worst, nd, R);
      std::fflush(stderr);
    }
  }
  hipLaunchKernelGGL(k_from_z<T>, dim3(grid1d(tot)), blk, 0, st, x, reinterpret_cast<CT*>(xv), tot);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int r = 0; r < R; ++r) {
    res[r].iterations = iters[r];
    res[r].true_rel_res = bnorm[r] > 0 ? rnorm[r] / bnorm[r] : 0.0;
    res[r].converged = res[r].true_rel_res <= rtol;
    res[r].time_s = secs;
    res[r].reorth = reorth[r];
    res[r].cycles = cycles[r];
  }
  return 0;
}

// ------------------------------------------------ device pair assembly --
// Galerkin blocks between separated particles (Sec. II.A entries of
// Z^{pq}, exterior medium), FP64.  For observation points a and source
// points b the sums
//   SG[a][f][n] = sum_b w_b g(R_ab) v_b[f][n]            f: psi x,y,z, div
//   SH[a][f][n] = sum_b w_b h(R_ab) v_b[f'][n]           f': psi, psi x r_b
// with g = exp(-jkR)/(4 pi R) and grad g = h (r_a - r_b), are a complex-by-
// real matrix product whose left operand is generated on the fly: an FP64
// MFMA GEMM (16 observation points x 4 source points per step, the lane
// that holds A[i][k] evaluates g and h for that point pair).  Lane layout of
// v_mfma_f64_16x16x4f64: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k,
// result register v of lane l is row l/16 + 4v, column l % 16.  A second pass
// contracts the sums with the observation functions into T and K.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kPairWaves = 4;
constexpr int kPairTPW = 8;  // column tiles per wave: 10 * npad / 16 <= 32, i.e. N <= 48

struct PairJobDev {
  const double* qa;  // [Qa][3] observation points
  const double* wa;  // [Qa] observation weights
  const double* va;  // [Qa][7][Na] observation values
  const double* qb;  // [Qb][3] source points (local to the source particle)
  const double* Vb;  // [Qb][ncol] source values with the source weight folded in
  double* acc;       // [Qa][ncol][2] sums (re, im)
  double ox, oy, oz; // source centre relative to the observation centre
  int Qa, Qb, Na;
};

__global__ __launch_bounds__(kPairWaves * 64) void k_pair_sums(const PairJobDev* __restrict__ jobs, int npad,
                                                                double k) {
  __shared__ double gh[2][kPairWaves][4][64];  // [buffer][b-step][g re, g im, h re, h im][lane]
  const PairJobDev J = jobs[blockIdx.y];
  const int a0 = blockIdx.x * 16;
  if (a0 >= J.Qa) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  const int ntile = 10 * npad / 16, ntg = 4 * npad / 16, ncol = 16 * ntile;
  const int a = a0 + i;
  double xa = 0, ya = 0, za = 0;
  if (a < J.Qa) {
    xa = J.qa[3 * a] - J.ox;
    ya = J.qa[3 * a + 1] - J.oy;
    za = J.qa[3 * a + 2] - J.oz;
  }
  f64x4 accr[kPairTPW], acci[kPairTPW];
#pragma unroll
  for (int t = 0; t < kPairTPW; ++t) {
    accr[t] = f64x4{0, 0, 0, 0};
    acci[t] = f64x4{0, 0, 0, 0};
  }
  const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
  int buf = 0;
  // each iteration covers 4 * kPairWaves source points: wave w evaluates the
  // kernel for b-step w into LDS, then every wave runs all kPairWaves steps
  for (int b0 = 0; b0 < J.Qb; b0 += 4 * kPairWaves, buf ^= 1) {
    {
      const int b = b0 + 4 * wave + kq;
      double gr = 0, gi = 0, hr = 0, hi = 0;
      if (a < J.Qa && b < J.Qb) {
        const double dx = xa - J.qb[3 * b], dy = ya - J.qb[3 * b + 1], dz = za - J.qb[3 * b + 2];
        const double R = sqrt(dx * dx + dy * dy + dz * dz);
        const double kR = k * R;
        double sn, cs;
        sincos(kR, &sn, &cs);
        const double inv = inv4pi / R, inv3 = inv / (R * R);
        gr = cs * inv;
        gi = -sn * inv;
        hr = -(cs + kR * sn) * inv3;
        hi = -(kR * cs - sn) * inv3;
      }
      gh[buf][wave][0][lane] = gr;
      gh[buf][wave][1][lane] = gi;
      gh[buf][wave][2][lane] = hr;
      gh[buf][wave][3][lane] = hi;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < kPairWaves; ++st) {
      const int b = b0 + 4 * st + kq;
      const double gr = gh[buf][st][0][lane], gi = gh[buf][st][1][lane];
      const double hr = gh[buf][st][2][lane], hi = gh[buf][st][3][lane];
      const double* __restrict__ vrow = J.Vb + (size_t)(b < J.Qb ? b : 0) * ncol;
#pragma unroll
      for (int t = 0; t < kPairTPW; ++t) {
        const int jt = wave + kPairWaves * t;
        if (jt < ntile) {
          const double bv = b < J.Qb ? vrow[jt * 16 + i] : 0.0;
          const bool isg = jt < ntg;
          accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(isg ? gr : hr, bv, accr[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(isg ? gi : hi, bv, acci[t], 0, 0, 0);
        }
      }
    }
    // the buffer written next iteration was last read before this barrier
  }
#pragma unroll
  for (int t = 0; t < kPairTPW; ++t) {
    const int jt = wave + kPairWaves * t;
    if (jt >= ntile) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ar = a0 + kq + 4 * v;  // FP64 16x16x4 result: register v of lane l is row l/16 + 4v
      if (ar < J.Qa) {
        double* o = J.acc + ((size_t)ar * ncol + jt * 16 + i) * 2;
        o[0] = accr[t][v];
        o[1] = acci[t][v];
      }
    }
  }
}

// T[m][n] = sum_a w_a (-jk psi_m . SG[0..2] + (j/k) div psi_m SG[3])
// K[m][n] = sum_a w_a (r_a x psi_m . SH[0..2] - psi_m . (SH[3..5] + SH[0..2] x offset))
// Block = (source function n, job); threads stride over a; 8 observation
// functions per pass.
constexpr int kPairMC = 8;
__global__ __launch_bounds__(kBlock) void k_pair_contract(const PairJobDev* __restrict__ jobs, int npad, double k,
                                                           double* __restrict__ TK) {
  const PairJobDev J = jobs[blockIdx.y];
  const int n = blockIdx.x;
  const int Na = J.Na, ncol = 10 * npad;
  __shared__ double red[kBlock / 64][4 * kPairMC];
  for (int m0 = 0; m0 < Na; m0 += kPairMC) {
    double acc[4 * kPairMC];  // T re, T im, K re, K im per m
#pragma unroll
    for (int q = 0; q < 4 * kPairMC; ++q) acc[q] = 0;
    for (int a = threadIdx.x; a < J.Qa; a += kBlock) {
      const double* s = J.acc + (size_t)a * ncol * 2;
      double g[4][2], h[6][2];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        g[f][0] = s[(f * npad + n) * 2];
        g[f][1] = s[(f * npad + n) * 2 + 1];
      }
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        h[f][0] = s[((4 + f) * npad + n) * 2];
        h[f][1] = s[((4 + f) * npad + n) * 2 + 1];
      }
      // psi_q x r_b with r_b measured from the observation centre
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double ux = h[0][c], uy = h[1][c], uz = h[2][c];
        h[3][c] += uy * J.oz - uz * J.oy;
        h[4][c] += uz * J.ox - ux * J.oz;
        h[5][c] += ux * J.oy - uy * J.ox;
      }
      const double w = J.wa[a];
      const double rx = J.qa[3 * a], ry = J.qa[3 * a + 1], rz = J.qa[3 * a + 2];
      const double* va = J.va + (size_t)a * 7 * Na;
#pragma unroll
      for (int mm = 0; mm < kPairMC; ++mm) {
        const int m = m0 + mm;
        if (m >= Na) break;
        const double px = va[m], py = va[Na + m], pz = va[2 * Na + m], dm = va[3 * Na + m];
        const double qx = ry * pz - rz * py, qy = rz * px - rx * pz, qz = rx * py - ry * px;  // r_a x psi_m
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const double vec = px * g[0][c] + py * g[1][c] + pz * g[2][c];
          const double dv = dm * g[3][c];
          const double ku = qx * h[0][c] + qy * h[1][c] + qz * h[2][c] - (px * h[3][c] + py * h[4][c] + pz * h[5][c]);
          // T: -jk vec + (j/k) dv  ->  (re, im) contributions
          if (c == 0) {
            acc[4 * mm + 1] += w * (-k * vec + dv / k);
            acc[4 * mm + 2] += w * ku;
          } else {
            acc[4 * mm + 0] += w * (k * vec - dv / k);
            acc[4 * mm + 3] += w * ku;
          }
        }
      }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 4 * kPairMC; ++q) {
      const double v = wave_sum(acc[q]);
      if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4 * kPairMC) {
      const int q = threadIdx.x, mm = q / 4, part = q % 4;
      const int m = m0 + mm;
      if (m < Na) {
        double v = 0;
        for (int w2 = 0; w2 < kBlock / 64; ++w2) v += red[w2][q];
        // TK layout per job: [2 (T, K)][Na][Na][2 (re, im)]
        const int which = part / 2, ri = part % 2;
        TK[(((size_t)blockIdx.y * 2 + which) * Na * Na + (size_t)m * Na + n) * 2 + ri] = v;
      }
    }
    __syncthreads();
  }
}

}  // namespace

Engine* make_engine(int precision) {
  if (precision == 1) return new EngineT<double>();
  return new EngineT<float>();
}

int gpu_pair_blocks(const std::vector<PairSamples>& cls, const std::vector<PairRequest>& req, double k,
                    std::vector<std::vector<cd>>& T, std::vector<std::vector<cd>>& K, std::string& err) {
  T.assign(req.size(), {});
  K.assign(req.size(), {});
  if (req.empty()) return 0;
  int N = -1;
  for (const auto& c : cls)
    if (c.val) N = std::max(N, c.N);
  const int npad = (N + 15) / 16 * 16;
  if (10 * npad / 16 > kPairWaves * kPairTPW) {
    err = "device pair assembly supports at most 48 functions per class";
    return -1;
  }
  const int ncol = 10 * npad;
  // per-class device samples
  struct Dev {
    DevMem qp, qw, val, Vb;
    int Q = 0;
  };
  std::vector<Dev> dev(cls.size());
  for (size_t c = 0; c < cls.size(); ++c) {
    const PairSamples& S = cls[c];
    if (!S.val) continue;
    if (S.N != N) {
      err = "pair assembly: classes differ in their number of functions";
      return -1;
    }
    const int Q = (int)S.qp->size();
    std::vector<double> qp((size_t)Q * 3), Vb((size_t)Q * ncol, 0.0);
    for (int q = 0; q < Q; ++q) {
      qp[3 * q] = (*S.qp)[q].x;
      qp[3 * q + 1] = (*S.qp)[q].y;
      qp[3 * q + 2] = (*S.qp)[q].z;
      const double w = (*S.qw)[q];
      const double* v = &(*S.val)[(size_t)q * 7 * N];
      double* o = &Vb[(size_t)q * ncol];
      for (int n = 0; n < N; ++n) {
        for (int f = 0; f < 4; ++f) o[f * npad + n] = w * v[f * N + n];
        for (int f = 0; f < 3; ++f) o[(4 + f) * npad + n] = w * v[f * N + n];
        for (int f = 0; f < 3; ++f) o[(7 + f) * npad + n] = w * v[(4 + f) * N + n];
      }
    }
    Dev& d = dev[c];
    d.Q = Q;
    auto put = [&](DevMem& m, const std::vector<double>& h) -> hipError_t {
      hipError_t e = m.alloc(h.size() * sizeof(double));
      if (e == hipSuccess) e = hipMemcpy(m.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
      return e;
    };
    HIP_TRY(put(d.qp, qp));
    HIP_TRY(put(d.qw, *S.qw));
    HIP_TRY(put(d.val, *S.val));
    HIP_TRY(put(d.Vb, Vb));
  }
  int Qmax = 0;
  for (const auto& d : dev) Qmax = std::max(Qmax, d.Q);
  const size_t per_job = (size_t)Qmax * ncol * 2;
  const int batch = (int)std::max<size_t>(1, std::min<size_t>(64, ((size_t)1 << 30) / (per_job * sizeof(double))));
  DevMem acc, jobs, tk;
  HIP_TRY(acc.alloc((size_t)batch * per_job * sizeof(double)));
  HIP_TRY(jobs.alloc((size_t)batch * sizeof(PairJobDev)));
  HIP_TRY(tk.alloc((size_t)batch * 2 * N * N * 2 * sizeof(double)));
  std::vector<double> htk((size_t)batch * 2 * N * N * 2);
  for (size_t j0 = 0; j0 < req.size(); j0 += batch) {
    const int nb = (int)std::min<size_t>(batch, req.size() - j0);
    std::vector<PairJobDev> hj(nb);
    int Qa_max = 0;
    for (int j = 0; j < nb; ++j) {
      const PairRequest& r = req[j0 + j];
      if (r.cp < 0 || r.cq < 0 || r.cp >= (int)cls.size() || r.cq >= (int)cls.size() || !cls[r.cp].val ||
          !cls[r.cq].val) {
        err = "pair assembly: class without samples";
        return -1;
      }
      const Dev &A = dev[r.cp], &B = dev[r.cq];
      PairJobDev& J = hj[j];
      J.qa = A.qp.as<double>();
      J.wa = A.qw.as<double>();
      J.va = A.val.as<double>();
      J.qb = B.qp.as<double>();
      J.Vb = B.Vb.as<double>();
      J.acc = acc.as<double>() + (size_t)j * per_job;
      J.ox = r.offset.x;
      J.oy = r.offset.y;
      J.oz = r.offset.z;
      J.Qa = A.Q;
      J.Qb = B.Q;
      J.Na = N;
      Qa_max = std::max(Qa_max, A.Q);
    }
    HIP_TRY(hipMemcpy(jobs.p, hj.data(), nb * sizeof(PairJobDev), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_pair_sums, dim3((Qa_max + 15) / 16, nb), dim3(kPairWaves * 64), 0, 0,
                       jobs.as<PairJobDev>(), npad, k);
    hipLaunchKernelGGL(k_pair_contract, dim3(N, nb), dim3(kBlock), 0, 0, jobs.as<PairJobDev>(), npad, k,
                       tk.as<double>());
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpy(htk.data(), tk.p, (size_t)nb * 2 * N * N * 2 * sizeof(double), hipMemcpyDeviceToHost));
    for (int j = 0; j < nb; ++j) {
      std::vector<cd>& Tj = T[j0 + j];
      std::vector<cd>& Kj = K[j0 + j];
      Tj.resize((size_t)N * N);
      Kj.resize((size_t)N * N);
      const double* base = &htk[(size_t)j * 2 * N * N * 2];
      for (int e = 0; e < N * N; ++e) {
        Tj[e] = cd(base[2 * e], base[2 * e + 1]);
        Kj[e] = cd(base[2 * (N * N + e)], base[2 * (N * N + e) + 1]);
      }
    }
  }
  return 0;
}

}  // namespace mlfma
