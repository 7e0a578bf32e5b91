// Three-phonon linewidths of a Gamma-point solid (one cell, N_q = 1, real
// eigenvectors E[component][mode]).
//
// Paper: Eq. phi3_proj with real eigenvectors, which for each mode mu is the
// matrix product V_mu = E^T (A_mu E) with the sparse
// A_mu[b][c] = sum_a Phi3_abc E_a,mu / sqrt(m_a m_b m_c); Eq. gamma, Eq. bose,
// Eq. broadening with the 2-sigma cut, as on the crystal path with N_q = 1.
//
// Kernels per batch of modes:
//   gp_avals   A_mu values on the fixed (b, c) pattern        (sparse x E)
//   gp_spmm    W_mu = A_mu E, row b of W from the ~15 entries of row b of A_mu
//   gp_gemm    V tile = E^T W_mu on a 64 x 64 (mu', mu'') tile, K = 3N, and the
//              FP64 cut / weight / |V|^2 epilogue reduced to one partial per
//              tile; tiles whose frequency ranges cannot meet the cut exit
//              before loading anything
//   gp_finish  fixed-order sum of the tile partials per mode
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "common.h"
#include "lw_common.h"

namespace kaldo {

constexpr int kGpTile = 64;
constexpr int kGpK = 16;
constexpr int kGpBatch = 64;

// E rounded to T; a non-finite entry raises kFlagNonFinite.
template <typename T>
__global__ void gp_round(long n, const double* __restrict__ src, T* __restrict__ dst,
                         int32_t* __restrict__ flags) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double x = src[k];
  dst[k] = (T)x;
  if (!(x - x == 0.0)) raise_flag(flags, kFlagNonFinite);
}

// Per mode: population and masks, and validation of omega (non-finite:
// kFlagNonFinite; imaginary with |nu| >= nu_min: kFlagImaginary).  The
// eigenvectors are checked where they are rounded to the contraction type.
__global__ void gp_prepare(int n, const double* __restrict__ omega,
                           double inv_kt_hbar, double nu_min, double* __restrict__ occ,
                           uint8_t* __restrict__ phys, uint8_t* __restrict__ sel, int sel_all,
                           int32_t* __restrict__ flags) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double w = omega[m];
  bool p = (w / kTwoPi) >= nu_min;
  phys[m] = p;
  occ[m] = p ? 1.0 / expm1(w * inv_kt_hbar) : 0.0;
  sel[m] = sel_all ? 1 : 0;
  if (!(w - w == 0.0)) raise_flag(flags, kFlagNonFinite);
  if (w < 0.0 && (-w / kTwoPi) >= nu_min) raise_flag(flags, kFlagImaginary);
}

__global__ void gp_select(const int32_t* __restrict__ subset, long n_subset, int n,
                          uint8_t* __restrict__ sel, int32_t* __restrict__ flags) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_subset) return;
  int m = subset[k];
  if (m >= 0 && m < n)
    sel[m] = 1;
  else
    raise_flag(flags, kFlagSubset);
}

// avals[j][k] = sum_{t in pattern k} coef_t E[a_t][mode m0 + j]  (FP64 sum)
template <typename T>
__global__ void gp_avals(int n, int n_bc, int m0, int nbatch, const int32_t* __restrict__ t_ptr,
                         const int32_t* __restrict__ t_a, const double* __restrict__ t_coef,
                         const double* __restrict__ E, T* __restrict__ avals) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)n_bc * nbatch) return;
  int j = k / n_bc, e = k % n_bc;
  int mu = m0 + j;
  double s = 0.0;
  for (int t = t_ptr[e]; t < t_ptr[e + 1]; ++t) s += t_coef[t] * E[(size_t)t_a[t] * n + mu];
  avals[k] = (T)s;
}

// W[j][b][c'] = sum_{k in row b} avals[j][k] Et[col_k][c']
template <typename T>
__global__ void gp_spmm(int n, int n_bc, int nbatch, const int32_t* __restrict__ row_ptr,
                        const int32_t* __restrict__ col, const T* __restrict__ avals,
                        const T* __restrict__ Et, T* __restrict__ W) {
  const int b = blockIdx.x;
  const int j = blockIdx.y;
  const T* av = avals + (size_t)j * n_bc;
  T* out = W + ((size_t)j * n + b) * n;
  const int k0 = row_ptr[b], k1 = row_ptr[b + 1];
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    T s = 0;
    for (int k = k0; k < k1; ++k) s += av[k] * Et[(size_t)col[k] * n + c];
    out[c] = s;
  }
}

// One 64x64 tile of V_mu = E^T W_mu with the fused FP64 epilogue.
template <typename T>
__global__ __launch_bounds__(256) void gp_gemm(LwParams p, int n, int m0, const T* __restrict__ Et,
                                               const T* __restrict__ W,
                                               const double* __restrict__ omega,
                                               const double* __restrict__ occ,
                                               const uint8_t* __restrict__ phys,
                                               const uint8_t* __restrict__ sel,
                                               double* __restrict__ partial, int n_tiles) {
  __shared__ T As[kGpK][kGpTile + 1];
  __shared__ T Bs[kGpK][kGpTile + 1];
  __shared__ double red[256];
  __shared__ int skip;
  const int tid = threadIdx.x;
  const int mu = m0 + blockIdx.z;
  const int i0 = blockIdx.y * kGpTile, j0 = blockIdx.x * kGpTile;
  const int tile_id = blockIdx.y * n_tiles + blockIdx.x;
  double* out = partial + (size_t)mu * n_tiles * n_tiles + tile_id;
  if (!sel[mu] || !phys[mu]) {
    if (tid == 0) *out = 0.0;
    return;
  }
  const double w = omega[mu];
  // Frequency ranges of the tile's physical partners; exact skip test.
  if (tid == 0) {
    double lo1 = 1e300, hi1 = -1e300, lo2 = 1e300, hi2 = -1e300;
    for (int k = 0; k < kGpTile; ++k) {
      int a = i0 + k, b = j0 + k;
      if (a < n && phys[a]) { lo1 = fmin(lo1, omega[a]); hi1 = fmax(hi1, omega[a]); }
      if (b < n && phys[b]) { lo2 = fmin(lo2, omega[b]); hi2 = fmax(hi2, omega[b]); }
    }
    int sk = 1;
    if (lo1 <= hi1 && lo2 <= hi2) {
      // x+ = w + w1 - w2 and x- = w - w1 - w2 over the tile, |x| < 2 sigma
      double reach = 2.0 * p.sig_fixed * (1.0 + 1e-12) + 1e-9;
      double xp_lo = w + lo1 - hi2, xp_hi = w + hi1 - lo2;
      double xm_lo = w - hi1 - hi2, xm_hi = w - lo1 - lo2;
      bool can_p = xp_lo < reach && xp_hi > -reach;
      bool can_m = xm_lo < reach && xm_hi > -reach;
      sk = !(can_p || can_m);
    }
    skip = sk;
  }
  __syncthreads();
  if (skip) {
    if (tid == 0) *out = 0.0;
    return;
  }
  const T* Wm = W + (size_t)blockIdx.z * n * n;
  const int tr = tid / 16, tc = tid % 16;  // 4x4 outputs per thread
  T acc[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) acc[a][b] = 0;
  for (int k0 = 0; k0 < n; k0 += kGpK) {
    for (int idx = tid; idx < kGpK * kGpTile; idx += 256) {
      int kk = idx / kGpTile, cc = idx % kGpTile;
      int k = k0 + kk;
      As[kk][cc] = (k < n && i0 + cc < n) ? Et[(size_t)k * n + i0 + cc] : (T)0;
      Bs[kk][cc] = (k < n && j0 + cc < n) ? Wm[(size_t)k * n + j0 + cc] : (T)0;
    }
    __syncthreads();
    for (int kk = 0; kk < kGpK; ++kk) {
      T a[4], b[4];
      for (int r = 0; r < 4; ++r) a[r] = As[kk][tr + 16 * r];
      for (int r = 0; r < 4; ++r) b[r] = Bs[kk][tc + 16 * r];
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
    }
    __syncthreads();
  }
  double sum = 0.0;
  for (int r = 0; r < 4; ++r) {
    int i = i0 + tr + 16 * r;
    if (i >= n || !phys[i]) continue;
    const double w1 = omega[i], n1 = occ[i];
    for (int c = 0; c < 4; ++c) {
      int j = j0 + tc + 16 * c;
      if (j >= n || !phys[j]) continue;
      double wt = pair_weight(p, w, w1, omega[j], n1, occ[j], p.sig_fixed, p.sig_fixed);
      if (wt == 0.0) continue;
      double v = (double)acc[r][c];
      sum += v * v * wt;
    }
  }
  red[tid] = sum;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) *out = red[0];
}

__global__ void gp_finish(int n, int n_tiles2, const double* __restrict__ partial,
                          const uint8_t* __restrict__ phys, const uint8_t* __restrict__ sel,
                          double* __restrict__ gamma) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n || !sel[m]) return;
  double acc = 0.0;
  for (int t = 0; t < n_tiles2; ++t) acc += partial[(size_t)m * n_tiles2 + t];
  gamma[m] = phys[m] ? kPrefactor * acc : 0.0;
}

struct GammaWs {
  size_t off_occ, off_phys, off_sel, off_et, off_av, off_w, off_partial, off_rest, total;
};

size_t gm_workspace_bytes(const kaldo_crystal* c, int prec);
int run_gm(const kaldo_crystal* c, const LwParams& p, const double* omega, const double* evec,
           const double* occ, const uint8_t* phys, const uint8_t* sel, unsigned char* ws,
           int prec, double* gamma, hipStream_t st);

bool gm_supported(const kaldo_crystal* c);

static bool use_mfma(const kaldo_crystal* c, int prec) {
  if (prec == KALDO_FP64 || !gm_supported(c)) return false;
  if (prec == KALDO_BF16X3) return true;
  const char* f = std::getenv("KALDO_FORCE_GENERIC");
  return !(f && f[0] == '1');
}

static GammaWs gamma_ws(const kaldo_crystal* c, int prec) {
  const size_t n = c->nb3;
  const size_t es = prec == KALDO_FP64 ? 8 : 4;
  const size_t nt = (n + kGpTile - 1) / kGpTile;
  GammaWs w;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  w.off_occ = take(8 * n);
  w.off_phys = take(n);
  w.off_sel = take(n);
  w.off_rest = o;
  w.off_et = take(es * n * n);
  w.off_av = take(es * (size_t)c->gamma.n_bc * kGpBatch);
  w.off_w = take(es * n * n * kGpBatch);
  w.off_partial = take(8 * n * nt * nt);
  w.total = o;
  if (prec != KALDO_FP64 && gm_supported(c))
    w.total = std::max(w.total, w.off_rest + gm_workspace_bytes(c, prec));
  return w;
}

template <typename T>
static int run_gamma(const kaldo_crystal* c, const double* omega, const double* evec, double Tk,
                     const kaldo_broadening* b, const int32_t* subset, int64_t n_subset,
                     unsigned char* ws, const GammaWs& g, int prec, double* gamma,
                     hipStream_t st) {
  const int n = c->nb3;
  const int nt = (n + kGpTile - 1) / kGpTile;
  double* occ = reinterpret_cast<double*>(ws + g.off_occ);
  uint8_t* phys = ws + g.off_phys;
  uint8_t* sel = ws + g.off_sel;
  T* Et = reinterpret_cast<T*>(ws + g.off_et);
  T* av = reinterpret_cast<T*>(ws + g.off_av);
  T* W = reinterpret_cast<T*>(ws + g.off_w);
  double* partial = reinterpret_cast<double*>(ws + g.off_partial);
  KALDO_LAUNCH("gp_prepare", gp_prepare, dim3((n + 255) / 256), dim3(256), 0, st, n, omega,
               kHbar / (kKb * Tk), b->nu_min_thz, occ, phys, sel, subset ? 0 : 1, c->d_flags);
  if (subset && n_subset > 0)
    KALDO_LAUNCH("gp_select", gp_select, dim3((n_subset + 255) / 256), dim3(256), 0, st, subset,
                 (long)n_subset, n, sel, c->d_flags);
  int32_t mesh1[3] = {1, 1, 1};
  LwParams p = make_params(c, mesh1, Tk, b);
  if (use_mfma(c, prec))
    return run_gm(c, p, omega, evec, occ, phys, sel, ws + g.off_rest, prec, gamma, st);
  long nn = (long)n * n;
  KALDO_LAUNCH("gp_round", gp_round<T>, dim3((nn + 255) / 256), dim3(256), 0, st, nn, evec, Et,
               c->d_flags);
  for (int m0 = 0; m0 < n; m0 += kGpBatch) {
    int nb = std::min(kGpBatch, n - m0);
    long na = (long)c->gamma.n_bc * nb;
    KALDO_LAUNCH("gp_avals", gp_avals<T>, dim3((na + 255) / 256), dim3(256), 0, st, n, c->gamma.n_bc, m0,
                       nb, c->gamma.t_ptr, c->gamma.t_a, c->gamma.t_coef, evec, av);
    KALDO_LAUNCH("gp_spmm", gp_spmm<T>, dim3(n, nb), dim3(256), 0, st, n, c->gamma.n_bc, nb,
                       c->gamma.row_ptr, c->gamma.col, av, Et, W);
    KALDO_LAUNCH("gp_gemm", gp_gemm<T>, dim3(nt, nt, nb), dim3(256), 0, st, p, n, m0, Et, W, omega, occ,
                       phys, sel, partial, nt);
  }
  KALDO_LAUNCH("gp_finish", gp_finish, dim3((n + 255) / 256), dim3(256), 0, st, n, nt * nt, partial, phys,
                     sel, gamma);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

}  // namespace kaldo

using namespace kaldo;

extern "C" size_t kaldo_linewidths_gamma_workspace(const kaldo_crystal* c, int32_t precision) {
  if (!c || c->n_rep != 1) return 0;
  return gamma_ws(c, precision).total;
}

extern "C" int kaldo_linewidths_gamma(const kaldo_crystal* c, const double* omega,
                                      const double* evec, double temperature,
                                      const kaldo_broadening* b, int32_t precision,
                                      const int32_t* modes_subset, int64_t n_subset,
                                      void* workspace, size_t workspace_bytes, double* gamma,
                                      void* stream) {
  KALDO_REQUIRE(c && omega && evec && b && gamma, "kaldo_linewidths_gamma: NULL argument");
  KALDO_REQUIRE(c->n_rep == 1, "kaldo_linewidths_gamma: the cell must have a single replica");
  KALDO_REQUIRE(std::isfinite(temperature) && temperature > 0,
                "kaldo_linewidths_gamma: temperature <= 0");
  int rc = check_broadening(b, false);
  if (rc) return rc;
  KALDO_REQUIRE(precision == KALDO_FP64 || precision == KALDO_FP32 || precision == KALDO_BF16X3,
                "kaldo_linewidths_gamma: unknown precision");
  KALDO_REQUIRE(n_subset >= 0 && (n_subset == 0 || modes_subset),
                "kaldo_linewidths_gamma: bad subset");
  if (precision == KALDO_BF16X3 && !gm_supported(c)) {
    set_error("kaldo_linewidths_gamma: BF16X3 needs the MFMA path, whose SpMM tile does not fit LDS here");
    return KALDO_EUNSUPPORTED;
  }
  GammaWs g = gamma_ws(c, precision);
  KALDO_REQUIRE(workspace && workspace_bytes >= g.total, "kaldo_linewidths_gamma: workspace too small");
  if (modes_subset && n_subset == 0) return KALDO_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto* ws = static_cast<unsigned char*>(workspace);
  if (precision == KALDO_FP64)
    return run_gamma<double>(c, omega, evec, temperature, b, modes_subset, n_subset, ws, g,
                             precision, gamma, st);
  return run_gamma<float>(c, omega, evec, temperature, b, modes_subset, n_subset, ws, g, precision,
                          gamma, st);
}
