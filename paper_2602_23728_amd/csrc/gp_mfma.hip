// Gamma-point projection on the matrix cores.
//
// For each mode mu the vertex matrix is V_mu = E^T W_mu with W_mu = A_mu E
// (paper: Eq. phi3_proj with real eigenvectors).  When Phi3 is symmetric in
// its last two slots V_mu is symmetric, so only tiles (I, J) with I <= J of
// the 128 x 128 tiling are computed; an off-diagonal tile then stands for
// both orders of the partner pair, and its epilogue adds w(mu', mu'') +
// w(mu'', mu').  Without that symmetry every tile (I, J) is computed with the
// weight of its own order.  Tiles whose partner frequencies cannot meet the
// 2-sigma cut (in either order, for the symmetric form) exit before any
// load (exact interval test).
//
// Operands live in HBM transposed, k-contiguous: ET[m][k] = E[k][m] and
// WT[n][k] = W_mu[k][n], padded to a multiple of 128 with zeros.
//   FP32 form:  v_mfma_f32_16x16x4_f32 on FP32 operands.
//   BF16x3:     x = hi + lo with hi = bf16(x), lo = bf16(x - hi); each product
//               is hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with
//               FP32 accumulation (lo*lo dropped).
// Workgroup: 256 threads = 4 waves in a 2 x 2 arrangement, each wave owning a
// 64 x 64 block of the tile as 4 x 4 MFMA 16 x 16 accumulators.  The K loop
// stages 128 x KT slices of both operands through LDS.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "lw_common.h"

namespace kaldo {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;

constexpr int kMT = 128;   // output tile edge
constexpr int kMBatch = 512;  // modes per launch

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// ET (FP32 or bf16 hi/lo) from E (FP64, [k][m]); zero padding beyond n.  A
// non-finite entry of E raises kFlagNonFinite.
__global__ void gm_prep_et(int n, int np, const double* __restrict__ E, float* __restrict__ et32,
                           __bf16* __restrict__ eth, __bf16* __restrict__ etl,
                           int32_t* __restrict__ flags) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)np * np) return;
  const int m = idx / np, k = idx % np;
  const double x = (m < n && k < n) ? E[(size_t)k * n + m] : 0.0;
  if (!(x - x == 0.0)) raise_flag(flags, kFlagNonFinite);
  const float v = (float)x;
  if (et32) et32[idx] = v;
  if (eth) {
    __bf16 h, l;
    split_bf16(v, h, l);
    eth[idx] = h;
    etl[idx] = l;
  }
}

// E in FP32 with rows k-major (e32[k][m] = E[k][m], n x n): the SpMM stages
// its rows from this copy.
__global__ void gm_prep_e(int n, const double* __restrict__ E, float* __restrict__ e32) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (long)n * n) e32[idx] = (float)E[idx];
}

// A_mu values in FP32 for modes m0 .. m0 + nb - 1, in the ELL layout the
// SpMM reads with coalesced loads: the value of slot t of row b for mode j
// is avE[((t * kMBatch / 4 + j / 4) * np + b) * 4 + j % 4] (zero for the
// padding slots and for rows b >= n).  A workgroup takes slot t, 16 rows and
// 256 modes: the sums run with the modes across the threads (coalesced
// reads of E's rows), the tile is transposed through LDS, and each group of
// four modes is written as one run of 16 rows x 4 values.
constexpr int kAvRows = 16;
__global__ __launch_bounds__(256) void gm_avals(int n, int np, int max_row, int m0, int nb,
                                                const int32_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ t_ptr,
                                                const int32_t* __restrict__ t_a,
                                                const double* __restrict__ t_coef,
                                                const double* __restrict__ E,
                                                float* __restrict__ avE) {
  __shared__ float tile[kAvRows][256 + 1];
  const int t = blockIdx.x, b0 = blockIdx.y * kAvRows, jh = blockIdx.z * 256;
  const int tid = threadIdx.x;
  const int j = jh + tid;  // this thread's mode in the batch
  for (int rb = 0; rb < kAvRows; ++rb) {
    const int b = b0 + rb;
    double s = 0.0;
    if (j < nb && b < n) {
      const int e = row_ptr[b] + t;
      if (e < row_ptr[b + 1])
        for (int u = t_ptr[e]; u < t_ptr[e + 1]; ++u) s += t_coef[u] * E[(size_t)t_a[u] * n + m0 + j];
    }
    tile[rb][tid] = (float)s;
  }
  __syncthreads();
  // 64 groups of four modes, each a run of kAvRows x 4 floats
  for (int idx = tid; idx < 64 * kAvRows * 4; idx += 256) {
    const int jq = idx / (kAvRows * 4), w = idx % (kAvRows * 4), rb = w / 4, r = w % 4;
    avE[(((size_t)t * (kMBatch / 4) + jh / 4 + jq) * np + b0 + rb) * 4 + r] = tile[rb][4 * jq + r];
  }
}

// WT[j][c'][b] = sum_{k in row b} av[j][k] E[col_k][c'] for a tile of
// kSpmmRows rows b and 64 columns c', all modes j of the batch.  The E rows
// the tile touches (its unique column list) are staged once in LDS; each
// mode's 32 x 64 result is transposed through LDS so WT rows are written
// contiguously.  FP32 products and sums; the BF16x3 form stores hi/lo.
// Frequency range [lo, hi] of the physical modes of each 128-wide block
// (lo > hi for a block without any).
__global__ void gm_block_ranges(int n, int nt, const double* __restrict__ omega,
                                const uint8_t* __restrict__ phys, double* __restrict__ brange) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nt) return;
  double lo = 1e300, hi = -1e300;
  for (int k = 0; k < kMT; ++k) {
    const int a = I * kMT + k;
    if (a < n && phys[a]) {
      lo = fmin(lo, omega[a]);
      hi = fmax(hi, omega[a]);
    }
  }
  brange[2 * I] = lo;
  brange[2 * I + 1] = hi;
}

// Whether tile (I, J) of mode frequency w can hold a pair that meets the
// 2-sigma cut (exact interval test on the block ranges); for the symmetric
// form (I <= J) in either order of the pair.
__device__ __forceinline__ bool gm_tile_live(const LwParams& p, double w, const double* brange,
                                             int I, int J, bool sym) {
  const double lo1 = brange[2 * I], hi1 = brange[2 * I + 1];
  const double lo2 = brange[2 * J], hi2 = brange[2 * J + 1];
  if (!(lo1 <= hi1 && lo2 <= hi2)) return false;
  const double reach = 2.0 * p.sig_fixed * (1.0 + 1e-12) + 1e-9;
  auto can = [&](double l1, double h1, double l2, double h2) {
    const bool cp = (w + l1 - h2) < reach && (w + h1 - l2) > -reach;
    const bool cm = (w - h1 - h2) < reach && (w - l1 - l2) > -reach;
    return cp || cm;
  };
  return can(lo1, hi1, lo2, hi2) || (sym && I != J && can(lo2, hi2, lo1, hi1));
}

// need[jb][J] = 1 when some live tile (I, J) of mode m0 + jb reads the W
// columns of block J (I <= J for the symmetric form, every I otherwise).
__global__ void gm_need(LwParams p, int nt, int m0, int nb, const double* __restrict__ omega,
                        const uint8_t* __restrict__ phys, const uint8_t* __restrict__ sel,
                        const double* __restrict__ brange, uint8_t* __restrict__ need) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb * nt) return;
  const int jb = k / nt, J = k % nt;
  const int mu = m0 + jb;
  bool any = false;
  const bool sym = p.half != 0;
  if (sel[mu] && phys[mu])
    for (int I = 0; I < (sym ? J + 1 : nt); ++I) any = any || gm_tile_live(p, omega[mu], brange, I, J, sym);
  need[k] = any ? 1 : 0;
}

struct GmTileInfo {
  int ti, tj;
};

// t-th tile: of the upper triangle (ti <= tj) for the symmetric form, of the
// full nt x nt tiling otherwise; row-major.
__host__ __device__ inline int gm_tile_count(int nt, bool sym) { return sym ? nt * (nt + 1) / 2 : nt * nt; }
__device__ __forceinline__ GmTileInfo gm_tile(int t, int nt, bool sym) {
  if (!sym) return {t / nt, t % nt};
  int ti = 0, rem = t;
  while (rem >= nt - ti) {
    rem -= nt - ti;
    ++ti;
  }
  return {ti, ti + rem};
}

// Compacted list of the live (mode, tile) pairs of a batch, in (mode, tile)
// order: list[k] = jb * n_tri + t.  One workgroup, fixed-order scan.
__global__ __launch_bounds__(1024) void gm_live_list(LwParams p, int nt, int n_tri, int n,
                                                     const double* __restrict__ omega,
                                                     const uint8_t* __restrict__ phys,
                                                     const uint8_t* __restrict__ sel,
                                                     const double* __restrict__ brange,
                                                     int32_t* __restrict__ lists) {
  // one workgroup per batch of kMBatch modes; batch b's list starts at
  // lists + b (kMBatch n_tri + 1), its count is the region's last entry
  __shared__ int wave_tot[16];
  __shared__ int carry;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = (int)blockIdx.x * kMBatch, nb = min(kMBatch, n - m0);
  int32_t* list = lists + (size_t)blockIdx.x * ((size_t)kMBatch * n_tri + 1);
  int32_t* count = list + (size_t)kMBatch * n_tri;
  if (tid == 0) carry = 0;
  __syncthreads();
  const int total = nb * n_tri;
  for (int base = 0; base < total; base += 1024) {
    const int k = base + tid;
    int f = 0;
    if (k < total) {
      const int jb = k / n_tri, t = k % n_tri;
      const int mu = m0 + jb;
      if (sel[mu] && phys[mu]) {
        const GmTileInfo tt = gm_tile(t, nt, p.half != 0);
        f = gm_tile_live(p, omega[mu], brange, tt.ti, tt.tj, p.half != 0) ? 1 : 0;
      }
    }
    int incl = f;
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wave_tot[wv] = incl;
    __syncthreads();
    int o = carry, tot = 0;
    for (int w = 0; w < 16; ++w) {
      o += (w < wv) ? wave_tot[w] : 0;
      tot += wave_tot[w];
    }
    if (f) list[o + incl - 1] = k;
    __syncthreads();
    if (tid == 0) carry += tot;
    __syncthreads();
  }
  if (tid == 0) *count = carry;
}

__global__ void gm_zero(long n, double* __restrict__ x) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) x[k] = 0.0;
}

constexpr int kSpmmCols = 64;            // columns c' per workgroup
constexpr int kSpmmLds = kSpmmCols + 4;  // LDS row stride of the staged E rows (floats)
constexpr int kSpmmModes = 16;           // modes per workgroup
// WT[j][c'][b] = sum_{k in row b} A_mu_j[b][col_k] E[col_k][c'], for a tile of
// kSpmmRows rows (one per lane), kSpmmCols columns (16 per wave) and
// kSpmmModes modes.  The tile's E rows are staged in LDS (FP32); each lane
// walks its row's entries once per group of 4 columns and updates 4 x 16
// accumulators per entry.  Writes are contiguous along b.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void gm_spmm(int n, int np, int nb, int n_rtiles, int max_row,
                                               const int32_t* __restrict__ col_ell,
                                               const int32_t* __restrict__ tile_u_ptr,
                                               const int32_t* __restrict__ tile_u,
                                               const float* __restrict__ avE,
                                               const float* __restrict__ e32,
                                               float* __restrict__ wt32, __bf16* __restrict__ wth,
                                               __bf16* __restrict__ wtl, int nt,
                                               const uint8_t* __restrict__ need) {
  extern __shared__ float4 es4[];
  // [n_u][kSpmmLds]: rows padded by 16 bytes, so lanes reading the same
  // columns of different rows fall in different banks
  float* es = reinterpret_cast<float*>(es4);
  const int rt = blockIdx.x, c0 = blockIdx.y * kSpmmCols, j0 = blockIdx.z * kSpmmModes;
  {
    // columns no live GEMM tile of these modes reads are not computed
    bool any = false;
    for (int j = 0; j < kSpmmModes && j0 + j < nb; ++j) any = any || need[(j0 + j) * nt + c0 / kMT];
    if (!any) return;
  }
  const int b0 = rt * kSpmmRows;
  const bool has_rows = rt < n_rtiles;  // row tiles past the last row of A are zero
  const int u0 = has_rows ? tile_u_ptr[rt] : 0;
  const int n_u = has_rows ? tile_u_ptr[rt + 1] - u0 : 0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int idx = tid; idx < n_u * kSpmmCols; idx += 256) {
    const int u = idx / kSpmmCols, x = idx % kSpmmCols;
    es[u * kSpmmLds + x] = (c0 + x < n) ? e32[(size_t)tile_u[u0 + u] * n + c0 + x] : 0.0f;
  }
  __syncthreads();
  if (n_u == 0) {
    // no entries in these rows: W is zero there
    for (int idx = tid; idx < kSpmmModes * kSpmmCols * kSpmmRows; idx += 256) {
      const int j = idx / (kSpmmCols * kSpmmRows), x = (idx / kSpmmRows) % kSpmmCols, bb = idx % kSpmmRows;
      if (j0 + j >= nb) continue;
      const size_t g = ((size_t)(j0 + j) * np + c0 + x) * np + b0 + bb;
      if (wt32) wt32[g] = 0.0f;
      if (wth) {
        wth[g] = (__bf16)0.0f;
        wtl[g] = (__bf16)0.0f;
      }
    }
    return;
  }
  const int b = b0 + lane;
  // every row takes max_row slots (padding slots hold zero values and read
  // staged row 0); the A values of slot t for the workgroup's 16 modes are
  // four 16-byte loads that are contiguous across the wave's lanes
  const float4* av4 = reinterpret_cast<const float4*>(avE) + (size_t)(j0 / 4) * np + b;
  // each wave: 16 columns in two passes of 8 (8 x 16 accumulators), so every
  // nonzero's 16 mode values are loaded twice per column tile
  constexpr int XW = 8;
  for (int xc = 0; xc < kSpmmCols / 4 / XW; ++xc) {
    const int x0 = wv * (kSpmmCols / 4) + XW * xc;
    float acc[XW][kSpmmModes];
#pragma unroll
    for (int x = 0; x < XW; ++x)
#pragma unroll
      for (int j = 0; j < kSpmmModes; ++j) acc[x][j] = 0.0f;
    for (int t = 0; t < max_row; ++t) {
      const float4* ep = reinterpret_cast<const float4*>(&es[col_ell[(size_t)t * n + min(b, n - 1)] * kSpmmLds + x0]);
      const float4 e0 = ep[0], e1 = ep[1];
      const float4* ap = av4 + (size_t)t * (kMBatch / 4) * np;
      float a[kSpmmModes];
#pragma unroll
      for (int q = 0; q < kSpmmModes / 4; ++q) {
        const float4 v = ap[(size_t)q * np];
        a[4 * q] = v.x;
        a[4 * q + 1] = v.y;
        a[4 * q + 2] = v.z;
        a[4 * q + 3] = v.w;
      }
#pragma unroll
      for (int j = 0; j < kSpmmModes; ++j) {
        acc[0][j] += a[j] * e0.x;
        acc[1][j] += a[j] * e0.y;
        acc[2][j] += a[j] * e0.z;
        acc[3][j] += a[j] * e0.w;
        acc[4][j] += a[j] * e1.x;
        acc[5][j] += a[j] * e1.y;
        acc[6][j] += a[j] * e1.z;
        acc[7][j] += a[j] * e1.w;
      }
    }
#pragma unroll
    for (int j = 0; j < kSpmmModes; ++j) {
      if (j0 + j >= nb) break;
#pragma unroll
      for (int x = 0; x < XW; ++x) {
        const size_t g = ((size_t)(j0 + j) * np + c0 + x0 + x) * np + b;
        const float v = acc[x][j];
        // W is read back only by the GEMM of this batch, long after it has
        // left the caches: streaming (non-temporal) stores
        if (wt32) __builtin_nontemporal_store(v, &wt32[g]);
        if (wth) {
          __bf16 h, l;
          split_bf16(v, h, l);
          __builtin_nontemporal_store(h, &wth[g]);
          __builtin_nontemporal_store(l, &wtl[g]);
        }
      }
    }
  }
}

// Waves per SIMD the register allocation targets: three for the split form
// (measured 0.41 -> 0.38 ms per batch of the 512-atom glass), the compiler's
// choice (two) for FP32, where three measures the same and four spills.
template <bool SPLIT>
constexpr int gemm_waves_per_eu() {
  return SPLIT ? 3 : 1;
}

template <bool SPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gemm_waves_per_eu<SPLIT>()))) void gm_gemm(LwParams p, int n, int np, int m0, int n_tri,
                                               const float* __restrict__ et32,
                                               const __bf16* __restrict__ eth,
                                               const __bf16* __restrict__ etl,
                                               const float* __restrict__ wt32,
                                               const __bf16* __restrict__ wth,
                                               const __bf16* __restrict__ wtl,
                                               const double* __restrict__ omega,
                                               const double* __restrict__ occ,
                                               const uint8_t* __restrict__ phys,
                                               const int32_t* __restrict__ live_list,
                                               const int32_t* __restrict__ live_count,
                                               double* __restrict__ partial) {
  constexpr int KT = SPLIT ? 32 : 16;
  // LDS rows padded to stagger banks
  constexpr int LDA32 = KT + 4;        // floats (rows 16-byte aligned, reads conflict-free)
  constexpr int LDA16 = KT + 8;        // bf16 elements (row = 80 bytes)
  __shared__ __attribute__((aligned(16))) float sA32[SPLIT ? 1 : 2 * kMT * LDA32];  // two buffers
  __shared__ __attribute__((aligned(16))) float sB32[SPLIT ? 1 : 2 * kMT * LDA32];
  __shared__ __attribute__((aligned(16))) __bf16 sAh[SPLIT ? kMT * LDA16 : 8];
  __shared__ __attribute__((aligned(16))) __bf16 sAl[SPLIT ? kMT * LDA16 : 8];
  __shared__ __attribute__((aligned(16))) __bf16 sBh[SPLIT ? kMT * LDA16 : 8];
  __shared__ __attribute__((aligned(16))) __bf16 sBl[SPLIT ? kMT * LDA16 : 8];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nt = np / kMT;
  // workgroup k takes the k-th live (mode, tile) pair; the rest of the grid
  // (sized for every pair) exits at once
  if ((int)blockIdx.x >= *live_count) return;
  const int pair = live_list[blockIdx.x];
  const int jb = pair / n_tri, t = pair % n_tri;
  const GmTileInfo tt = gm_tile(t, nt, p.half != 0);
  const int mu = m0 + jb;
  const int i0 = tt.ti * kMT, j0 = tt.tj * kMT;
  const double w = omega[mu];
  double* out = partial + (size_t)mu * n_tri + t;

  const size_t wbase = (size_t)jb * np * np;
  const int wm = (wv >> 1) * 64, wn = (wv & 1) * 64;  // wave block inside the tile
  const int lr = lane & 15, lg = lane >> 4;
  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  // FP32 form: each thread moves NP 16-byte pieces of both operands per
  // slice.
  constexpr int PPR = KT / 4;  // 16-byte pieces per row (FP32 form)
  constexpr int NP = kMT * PPR / 256;  // pieces per thread
  static_assert(SPLIT || kMT * PPR == NP * 256, "whole pieces per thread");
  static_assert(SPLIT || KT % 16 == 0, "whole 16-byte groups per lane group");
  static_assert(SPLIT || NP == 2, "two 16-byte pieces of each operand per thread");
  // Staging registers are named scalars, not an array: the compiler moves a
  // private array indexed in a loop into LDS or scratch before unrolling, and
  // the prefetch then waits for its loads as soon as they are issued.
  if constexpr (!SPLIT) {
    // two LDS buffers: slice k0 + KT is fetched into registers and staged into
    // the idle buffer while slice k0 is multiplied; one barrier per slice
    uint4 pa0, pa1, pb0, pb1;
    const int r0 = tid / PPR, r1 = (tid + 256) / PPR, cc = (tid % PPR) * 4;
    const float* ga0 = et32 + (size_t)(i0 + r0) * np + cc;
    const float* ga1 = et32 + (size_t)(i0 + r1) * np + cc;
    const float* gb0 = wt32 + wbase + (size_t)(j0 + r0) * np + cc;
    const float* gb1 = wt32 + wbase + (size_t)(j0 + r1) * np + cc;
    const int sa0 = r0 * LDA32 + cc, sa1 = r1 * LDA32 + cc;
    pa0 = *reinterpret_cast<const uint4*>(ga0);
    pa1 = *reinterpret_cast<const uint4*>(ga1);
    pb0 = *reinterpret_cast<const uint4*>(gb0);
    pb1 = *reinterpret_cast<const uint4*>(gb1);
    *reinterpret_cast<uint4*>(&sA32[sa0]) = pa0;
    *reinterpret_cast<uint4*>(&sA32[sa1]) = pa1;
    *reinterpret_cast<uint4*>(&sB32[sa0]) = pb0;
    *reinterpret_cast<uint4*>(&sB32[sa1]) = pb1;
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < np; k0 += KT) {
      const bool more = k0 + KT < np;
      if (more) {
        pa0 = *reinterpret_cast<const uint4*>(ga0 + k0 + KT);
        pa1 = *reinterpret_cast<const uint4*>(ga1 + k0 + KT);
        pb0 = *reinterpret_cast<const uint4*>(gb0 + k0 + KT);
        pb1 = *reinterpret_cast<const uint4*>(gb1 + k0 + KT);
      }
      const float* A = sA32 + cur * kMT * LDA32;
      const float* B = sB32 + cur * kMT * LDA32;
      // K order inside the slice: lane group lg owns k in [KPL lg, KPL lg +
      // KPL) and MFMA step j of a 16-byte group pairs it with the group's
      // j-th value (the same on both operands), so a lane reads its k values
      // with one 16-byte LDS load per tile row and group
      constexpr int KPL = KT / 4;
#pragma unroll
      for (int h = 0; h < KPL / 4; ++h) {
        float4 a4[4], b4[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          a4[t] = *reinterpret_cast<const float4*>(&A[(wm + 16 * t + lr) * LDA32 + KPL * lg + 4 * h]);
          b4[t] = *reinterpret_cast<const float4*>(&B[(wn + 16 * t + lr) * LDA32 + KPL * lg + 4 * h]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int ta = 0; ta < 4; ++ta)
#pragma unroll
            for (int tb = 0; tb < 4; ++tb) {
              const float av = j == 0 ? a4[ta].x : j == 1 ? a4[ta].y : j == 2 ? a4[ta].z : a4[ta].w;
              const float bv = j == 0 ? b4[tb].x : j == 1 ? b4[tb].y : j == 2 ? b4[tb].z : b4[tb].w;
              acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[ta][tb], 0, 0, 0);
            }
      }
      if (more) {
        float* As = sA32 + (cur ^ 1) * kMT * LDA32;
        float* Bs = sB32 + (cur ^ 1) * kMT * LDA32;
        *reinterpret_cast<uint4*>(&As[sa0]) = pa0;
        *reinterpret_cast<uint4*>(&As[sa1]) = pa1;
        *reinterpret_cast<uint4*>(&Bs[sa0]) = pb0;
        *reinterpret_cast<uint4*>(&Bs[sa1]) = pb1;
      }
      __syncthreads();
      cur ^= 1;
    }
  } else {
    // one LDS buffer, the next slice prefetched into registers while the
    // current one is multiplied: each thread moves two 16-byte pieces (8 bf16)
    // of each of the four arrays per slice, as named scalars
    static_assert(kMT * (KT / 8) == 2 * 256, "two pieces per array and thread");
    const int r0 = tid / (KT / 8), r1 = (tid + 256) / (KT / 8), cc = (tid % (KT / 8)) * 8;
    const __bf16* pah0 = eth + (size_t)(i0 + r0) * np + cc;
    const __bf16* pah1 = eth + (size_t)(i0 + r1) * np + cc;
    const __bf16* pal0 = etl + (size_t)(i0 + r0) * np + cc;
    const __bf16* pal1 = etl + (size_t)(i0 + r1) * np + cc;
    const __bf16* pbh0 = wth + wbase + (size_t)(j0 + r0) * np + cc;
    const __bf16* pbh1 = wth + wbase + (size_t)(j0 + r1) * np + cc;
    const __bf16* pbl0 = wtl + wbase + (size_t)(j0 + r0) * np + cc;
    const __bf16* pbl1 = wtl + wbase + (size_t)(j0 + r1) * np + cc;
    const int l0 = r0 * LDA16 + cc, l1 = r1 * LDA16 + cc;
    uint4 xah0 = *reinterpret_cast<const uint4*>(pah0), xah1 = *reinterpret_cast<const uint4*>(pah1);
    uint4 xal0 = *reinterpret_cast<const uint4*>(pal0), xal1 = *reinterpret_cast<const uint4*>(pal1);
    uint4 xbh0 = *reinterpret_cast<const uint4*>(pbh0), xbh1 = *reinterpret_cast<const uint4*>(pbh1);
    uint4 xbl0 = *reinterpret_cast<const uint4*>(pbl0), xbl1 = *reinterpret_cast<const uint4*>(pbl1);
    *reinterpret_cast<uint4*>(&sAh[l0]) = xah0;
    *reinterpret_cast<uint4*>(&sAh[l1]) = xah1;
    *reinterpret_cast<uint4*>(&sAl[l0]) = xal0;
    *reinterpret_cast<uint4*>(&sAl[l1]) = xal1;
    *reinterpret_cast<uint4*>(&sBh[l0]) = xbh0;
    *reinterpret_cast<uint4*>(&sBh[l1]) = xbh1;
    *reinterpret_cast<uint4*>(&sBl[l0]) = xbl0;
    *reinterpret_cast<uint4*>(&sBl[l1]) = xbl1;
    __syncthreads();
    for (int k0 = 0; k0 < np; k0 += KT) {
      const bool more = k0 + KT < np;
      if (more) {
        const int kn = k0 + KT;
        xah0 = *reinterpret_cast<const uint4*>(pah0 + kn);
        xah1 = *reinterpret_cast<const uint4*>(pah1 + kn);
        xal0 = *reinterpret_cast<const uint4*>(pal0 + kn);
        xal1 = *reinterpret_cast<const uint4*>(pal1 + kn);
        xbh0 = *reinterpret_cast<const uint4*>(pbh0 + kn);
        xbh1 = *reinterpret_cast<const uint4*>(pbh1 + kn);
        xbl0 = *reinterpret_cast<const uint4*>(pbl0 + kn);
        xbl1 = *reinterpret_cast<const uint4*>(pbl1 + kn);
      }
      bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int ra = (wm + 16 * t + lr) * LDA16 + 8 * lg;
        const int rb = (wn + 16 * t + lr) * LDA16 + 8 * lg;
        ah[t] = *reinterpret_cast<const bf16x8*>(&sAh[ra]);
        al[t] = *reinterpret_cast<const bf16x8*>(&sAl[ra]);
        bh[t] = *reinterpret_cast<const bf16x8*>(&sBh[rb]);
        bl[t] = *reinterpret_cast<const bf16x8*>(&sBl[rb]);
      }
#pragma unroll
      for (int ta = 0; ta < 4; ++ta)
#pragma unroll
        for (int tb = 0; tb < 4; ++tb) {
          acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ta], bh[tb], acc[ta][tb], 0, 0, 0);
          acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ta], bl[tb], acc[ta][tb], 0, 0, 0);
          acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ta], bh[tb], acc[ta][tb], 0, 0, 0);
        }
      __syncthreads();  // every wave has read slice k0
      if (more) {
        *reinterpret_cast<uint4*>(&sAh[l0]) = xah0;
        *reinterpret_cast<uint4*>(&sAh[l1]) = xah1;
        *reinterpret_cast<uint4*>(&sAl[l0]) = xal0;
        *reinterpret_cast<uint4*>(&sAl[l1]) = xal1;
        *reinterpret_cast<uint4*>(&sBh[l0]) = xbh0;
        *reinterpret_cast<uint4*>(&sBh[l1]) = xbh1;
        *reinterpret_cast<uint4*>(&sBl[l0]) = xbl0;
        *reinterpret_cast<uint4*>(&sBl[l1]) = xbl1;
      }
      __syncthreads();  // slice k0 + KT visible
    }
  }

  // Epilogue: lane holds V[m = row0 + 4*lg + r][n = col0 + lr] of each 16 x 16 tile.
  // An off-diagonal tile of the symmetric form also stands for its mirror.
  const bool offdiag = p.half != 0 && tt.ti != tt.tj;
  const double s2 = 2.0 * p.sig_fixed;
  double sum = 0.0;
#pragma unroll
  for (int tb = 0; tb < 4; ++tb) {
    const int jn = j0 + wn + 16 * tb + lr;
    if (jn >= n || !phys[jn]) continue;
    const double w2 = omega[jn], n2 = occ[jn];
#pragma unroll
    for (int ta = 0; ta < 4; ++ta) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int im = i0 + wm + 16 * ta + 4 * lg + r;
        if (im >= n || !phys[im]) continue;
        const double w1 = omega[im];
        // quick reject: neither order of the pair is near the energy shell
        const double d1 = fabs(w + w1 - w2), d2 = fabs(w - w1 - w2);
        const double d3 = fabs(w + w2 - w1);
        const double lim = s2 * (1.0 + 1e-9) + 1e-9;
        if (d1 >= lim && d2 >= lim && (!offdiag || d3 >= lim)) continue;
        const double n1 = occ[im];
        double wt = pair_weight(p, w, w1, w2, n1, n2, p.sig_fixed, p.sig_fixed);
        if (offdiag) wt += pair_weight(p, w, w2, w1, n2, n1, p.sig_fixed, p.sig_fixed);
        if (wt == 0.0) continue;
        const double v = (double)acc[ta][tb][r];
        sum += v * v * wt;
      }
    }
  }
  // the operand buffers are idle after the K loop's last barrier; the
  // reduction reuses them (four FP32 workgroups then fit the 160 KB of LDS)
  double* red = SPLIT ? reinterpret_cast<double*>(sAh) : reinterpret_cast<double*>(sA32);
  static_assert(SPLIT || 2 * kMT * LDA32 * sizeof(float) >= 256 * sizeof(double), "room for the reduction");
  static_assert(!SPLIT || kMT * LDA16 * sizeof(__bf16) >= 256 * sizeof(double), "room for the reduction");
  red[tid] = sum;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) *out = red[0];
}

__global__ void gm_finish(int n, int n_tri, const double* __restrict__ partial,
                          const uint8_t* __restrict__ phys, const uint8_t* __restrict__ sel,
                          double* __restrict__ gamma) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n || !sel[m]) return;
  double acc = 0.0;
  for (int t = 0; t < n_tri; ++t) acc += partial[(size_t)m * n_tri + t];
  gamma[m] = phys[m] ? kPrefactor * acc : 0.0;
}

// The SpMM stages max_u rows of 64 floats in LDS.
bool gm_supported(const kaldo_crystal* c) {
  return (size_t)c->gamma.max_u * kSpmmLds * sizeof(float) <= 96 * 1024;
}

size_t gm_workspace_bytes(const kaldo_crystal* c, int prec) {
  const size_t n = c->nb3;
  const size_t np = (n + kMT - 1) / kMT * kMT;
  const size_t nt = np / kMT, n_tri = gm_tile_count((int)nt, c->bloch.sym_jk != 0);
  const bool split = prec == KALDO_BF16X3;
  size_t o = 0;
  auto take = [&](size_t bytes) { o += (bytes + 255) / 256 * 256; };
  take(np * np * 4);                       // et32
  take(n * n * 4);                         // e32 (the SpMM's rows, both forms)
  if (split) take(np * np * 2 * 2);         // eth, etl
  take((size_t)std::max(1, c->gamma.max_row) * np * kMBatch * 4);  // avals (ELL)
  take(split ? np * np * kMBatch * 2 * 2 : np * np * kMBatch * 4);  // W
  take(n * n_tri * 8);                     // partials
  take(nt * 2 * 8);                        // block frequency ranges
  take((size_t)kMBatch * nt);              // W column blocks needed per mode
  take((n + kMBatch - 1) / kMBatch * ((size_t)kMBatch * n_tri + 1) * 4);  // live lists and counts
  return o;
}

int run_gm(const kaldo_crystal* c, const LwParams& p, const double* omega, const double* evec,
           const double* occ, const uint8_t* phys, const uint8_t* sel, unsigned char* ws,
           int prec, double* gamma, hipStream_t st) {
  int32_t* flags = c->d_flags;
  const int n = c->nb3;
  const int np = (n + kMT - 1) / kMT * kMT;
  const int nt = np / kMT, n_tri = gm_tile_count(nt, p.half != 0);
  const bool split = prec == KALDO_BF16X3;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    unsigned char* r = ws + o;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  float* et32 = reinterpret_cast<float*>(take((size_t)np * np * 4));
  float* e32 = reinterpret_cast<float*>(take((size_t)n * n * 4));
  __bf16* eth = nullptr;
  __bf16* etl = nullptr;
  if (split) {
    eth = reinterpret_cast<__bf16*>(take((size_t)np * np * 2 * 2));  // hi and lo
    etl = eth + (size_t)np * np;
  }
  float* av = reinterpret_cast<float*>(take((size_t)std::max(1, c->gamma.max_row) * np * kMBatch * 4));
  float* wt32 = nullptr;
  __bf16* wth = nullptr;
  __bf16* wtl = nullptr;
  if (split) {
    wth = reinterpret_cast<__bf16*>(take((size_t)np * np * kMBatch * 4));
    wtl = wth + (size_t)np * np * kMBatch;
  } else {
    wt32 = reinterpret_cast<float*>(take((size_t)np * np * kMBatch * 4));
  }
  double* partial = reinterpret_cast<double*>(take((size_t)n * n_tri * 8));
  double* brange = reinterpret_cast<double*>(take((size_t)nt * 2 * 8));
  uint8_t* need = reinterpret_cast<uint8_t*>(take((size_t)kMBatch * nt));
  const int n_batch = (n + kMBatch - 1) / kMBatch;
  const size_t live_stride = (size_t)kMBatch * n_tri + 1;
  int32_t* live_lists = reinterpret_cast<int32_t*>(take((size_t)n_batch * live_stride * 4));
  const long n_part = (long)n * n_tri;
  KALDO_LAUNCH("gm_zero", gm_zero, dim3((unsigned)((n_part + 255) / 256)), dim3(256), 0, st, n_part, partial);
  const long nn = (long)np * np;
  KALDO_LAUNCH("gm_block_ranges", gm_block_ranges, dim3((nt + 63) / 64), dim3(64), 0, st, n, nt, omega,
               phys, brange);
  KALDO_LAUNCH("gm_prep_et", gm_prep_et, dim3((nn + 255) / 256), dim3(256), 0, st, n, np, evec,
               et32, eth, etl, flags);
  KALDO_LAUNCH("gm_prep_e", gm_prep_e, dim3((unsigned)(((long)n * n + 255) / 256)), dim3(256), 0, st, n,
               evec, e32);
  // the live (mode, tile) lists of every batch at once, one workgroup each
  KALDO_LAUNCH("gm_live_list", gm_live_list, dim3((unsigned)n_batch), dim3(1024), 0, st, p, nt, n_tri,
               n, omega, phys, sel, brange, live_lists);
  for (int m0 = 0; m0 < n; m0 += kMBatch) {
    const int nb = std::min(kMBatch, n - m0);
    int32_t* live_list = live_lists + (size_t)(m0 / kMBatch) * live_stride;
    int32_t* live_count = live_list + (size_t)kMBatch * n_tri;
    static_assert(kMBatch % 256 == 0, "whole 256-mode halves per batch");
    if (c->gamma.max_row > 0)
      KALDO_LAUNCH("gm_avals", gm_avals, dim3((unsigned)c->gamma.max_row, (unsigned)(np / kAvRows),
                   kMBatch / 256), dim3(256), 0, st, n, np, c->gamma.max_row, m0, nb,
                   c->gamma.row_ptr, c->gamma.t_ptr, c->gamma.t_a, c->gamma.t_coef, evec, av);
    KALDO_LAUNCH("gm_need", gm_need, dim3((nb * nt + 255) / 256), dim3(256), 0, st, p, nt, m0, nb, omega,
                 phys, sel, brange, need);
    const size_t spmm_lds = (size_t)c->gamma.max_u * kSpmmLds * sizeof(float);
    KALDO_LAUNCH("gm_spmm", gm_spmm, dim3(np / kSpmmRows, np / kSpmmCols, (nb + kSpmmModes - 1) / kSpmmModes),
                 dim3(256), spmm_lds, st, n, np, nb, c->gamma.n_rtiles, c->gamma.max_row,
                 c->gamma.col_ell, c->gamma.tile_u_ptr, c->gamma.tile_u, av, e32, wt32, wth, wtl, nt, need);
    if (split)
      KALDO_LAUNCH("gm_gemm_bf16x3", gm_gemm<true>, dim3(n_tri * nb), dim3(256), 0, st, p, n, np,
                   m0, n_tri, et32, eth, etl, wt32, wth, wtl, omega, occ, phys, live_list,
                   live_count, partial);
    else
      KALDO_LAUNCH("gm_gemm_fp32", gm_gemm<false>, dim3(n_tri * nb), dim3(256), 0, st, p, n, np,
                   m0, n_tri, et32, eth, etl, wt32, wth, wtl, omega, occ, phys, live_list,
                   live_count, partial);
  }
  KALDO_LAUNCH("gm_finish", gm_finish, dim3((n + 255) / 256), dim3(256), 0, st, n, n_tri, partial,
               phys, sel, gamma);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

}  // namespace kaldo
