// Isotope (mass-disorder) scattering of a crystal on a Gamma-centred mesh.
//
// Paper: Eq. isotope (Tamura's perturbation theory):
//   gamma_iso(q,s) = pi/(2 N_q) w^2 sum_{q' s'} delta(w - w')
//                    sum_i g_i |sum_a eta*_{ia}(q,s) eta_{ia}(q',s')|^2
// with the Cartesian sum inside the modulus (the form that does not depend on
// the orientation of the Cartesian axes), delta the smearing of Eq.
// broadening with its 2 sigma cut, partners and modes below nu_min excluded,
// and for the adaptive width sigma = max(floor, |v(q',s')| h / sqrt(12)) (the
// rate at which w - w' varies with the summed q').  gamma_iso is a linewidth
// in the convention of Eq. gamma, to which it adds (Eq. lifetime).
//
//   iso_prep     per mode: (w, sigma) record (w NaN below nu_min), eta
//                transposed to [q][mode][component], input checks
//   iso_sort     per branch the q-points in order of frequency (one
//                workgroup per branch, bitonic sort in LDS; larger meshes
//                keep the flat order)
//   iso_ranges   per (tile of partners in that order, branch): the frequency
//                range of its physical modes and their largest sigma
//   iso_kernel   one wave per four modes of a branch adjacent in that order
//                (nearly equal frequencies: they share each partner's loads):
//                per partner branch the run of tiles whose range can meet the
//                cut (found by binary search in the range table, in LDS),
//                lanes over the tile's partners, exact FP64 cut per mode and
//                partner, overlap and smearing in FP64, per-lane sums in tile
//                order, fixed wave reduction per mode
#include <algorithm>
#include <cmath>

#include "common.h"
#include "lw_common.h"

namespace kaldo {

constexpr int kIsoMaxBasis = 5;          // 3 N_b <= 16
constexpr size_t kIsoRangeLds = 48 << 10;  // bytes of range table kept in LDS

struct IsoParams {
  int nq, nb3, nb, blk, nblk;  // blk: partner q-points per tile (a multiple of 64)
  int shape, adaptive;
  double sig_fixed, sig_floor, h2, nu_min, scale;  // scale = pi / (2 N_q)
  double g[kIsoMaxBasis];
};

__global__ void iso_prep(IsoParams p, const double* __restrict__ omega, const double* __restrict__ vel,
                         const double* __restrict__ evec, double2* __restrict__ rec,
                         double2* __restrict__ inv, double2* __restrict__ etaT, int32_t* flags) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= p.nq * p.nb3) return;
  const int q = m / p.nb3, s = m - q * p.nb3;
  const double w = omega[m];
  const double v0 = vel[3 * (size_t)m], v1 = vel[3 * (size_t)m + 1], v2 = vel[3 * (size_t)m + 2];
  const bool phys = (w / kTwoPi) >= p.nu_min;
  double sig = p.sig_fixed;
  if (p.adaptive) sig = fmax(sqrt((v0 * v0 + v1 * v1 + v2 * v2) * p.h2 / 12.0), p.sig_floor);
  rec[m] = make_double2(phys ? w : __builtin_nan(""), sig);
  // 1/sigma and 1/(sqrt(pi) sigma) of the partner, once per mode
  inv[m] = make_double2(1.0 / sig, 1.0 / (kSqrtPi * sig));
  double chk = (w - w) + (v0 - v0) + (v1 - v1) + (v2 - v2);
  for (int j = 0; j < p.nb3; ++j) {
    const size_t src = (((size_t)q * p.nb3 + j) * p.nb3 + s) * 2;
    const double re = evec[src], im = evec[src + 1];
    chk += (re - re) + (im - im);
    etaT[(size_t)m * p.nb3 + j] = make_double2(re, im);
  }
  if (!(chk == 0.0)) raise_flag(flags, kFlagNonFinite);
  if (w < 0.0 && (-w / kTwoPi) >= p.nu_min) raise_flag(flags, kFlagImaginary);
}

// perm[s][i] = the i-th q-point of branch s in order of frequency: physical
// modes ascending (keys: the FP32 rounding of w, whose bits order like the
// values for w > 0, then q), the others last.  One workgroup per branch,
// bitonic sort of n2 = 2^k >= nq 64-bit keys in LDS; with sorted == 0 (too
// large a mesh for the LDS) the flat order.
__global__ __launch_bounds__(1024) void iso_sort(IsoParams p, int sorted, const double2* __restrict__ rec,
                                                 int32_t* __restrict__ perm) {
  extern __shared__ unsigned long long keys[];
  const int s = blockIdx.x;
  int32_t* out = perm + (size_t)s * p.nq;
  if (!sorted) {
    for (int i = threadIdx.x; i < p.nq; i += blockDim.x) out[i] = i;
    return;
  }
  int n2 = 1;
  while (n2 < p.nq) n2 <<= 1;
  for (int i = threadIdx.x; i < n2; i += blockDim.x) {
    unsigned long long k = ~0ull;
    if (i < p.nq) {
      const double w = rec[(size_t)i * p.nb3 + s].x;
      const unsigned hi = (w == w && w > 0.0) ? __float_as_uint((float)w) : 0xffffffffu;
      k = ((unsigned long long)hi << 32) | (unsigned)i;
    }
    keys[i] = k;
  }
  __syncthreads();
  for (int size = 2; size <= n2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const unsigned long long a = keys[i], b = keys[j];
          if ((a > b) == ((i & size) == 0)) {
            keys[i] = b;
            keys[j] = a;
          }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < p.nq; i += blockDim.x) out[i] = (int32_t)(keys[i] & 0xffffffffull);
}

// range[(s' * nblk + b)] = (lowest w, highest w, largest sigma) of the
// physical modes of branch s' in tile b of its order; an empty tile gets
// (+inf, -inf, 0).  Tiles run in frequency order, so lowest w does not
// decrease with b.
__global__ void iso_ranges(IsoParams p, const int32_t* __restrict__ perm,
                           const double2* __restrict__ rec, double* __restrict__ range) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p.nblk * p.nb3) return;
  const int s = k / p.nblk, b = k - s * p.nblk;
  double lo = INFINITY, hi = -INFINITY, smax = 0.0;
  const int i_end = min(p.nq, (b + 1) * p.blk);
  for (int i = b * p.blk; i < i_end; ++i) {
    const int q = perm[(size_t)s * p.nq + i];
    const double2 r = rec[(size_t)q * p.nb3 + s];
    if (r.x == r.x) {  // physical (not NaN)
      lo = fmin(lo, r.x);
      hi = fmax(hi, r.x);
      smax = fmax(smax, r.y);
    }
  }
  range[3 * (size_t)k] = lo;
  range[3 * (size_t)k + 1] = hi;
  range[3 * (size_t)k + 2] = smax;
}

// After the table: range[3 nblk nb3 + s'] = the largest sigma' over the tiles
// of branch s' (one thread per branch).
__global__ void iso_branch_smax(IsoParams p, double* __restrict__ range) {
  const int s = threadIdx.x;
  if (s >= p.nb3) return;
  double m = 0.0;
  for (int b = 0; b < p.nblk; ++b) m = fmax(m, range[3 * ((size_t)s * p.nblk + b) + 2]);
  range[3 * (size_t)p.nblk * p.nb3 + s] = m;
}

// Modes per wave: MPW modes of one branch at consecutive q-points (nearly the
// same frequency, so nearly the same live tiles and passing partners) share
// every partner's record and eigenvector load.
constexpr int kIsoMpw = 4;

template <int NB3>
__global__ __launch_bounds__(256) void iso_kernel(IsoParams p, const double2* __restrict__ rec,
                                                  const double2* __restrict__ inv,
                                                  const double2* __restrict__ etaT,
                                                  const double* __restrict__ range,
                                                  const int32_t* __restrict__ perm,
                                                  int accumulate, double* __restrict__ gamma) {
  constexpr int NB = NB3 / 3;
  constexpr int MPW = kIsoMpw;
  extern __shared__ double rng_lds[];  // the range table, [NB3][nblk][3], then [NB3] largest sigma'
  __shared__ double2 e0s[4][MPW][NB3];  // each wave's modes' eigenvectors
  const int n_rng = p.nblk * NB3 * 3 + NB3;
  for (int k = threadIdx.x; k < n_rng; k += blockDim.x) rng_lds[k] = range[k];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // wave -> (branch s, first position in the branch's frequency order):
  // waves of one branch are consecutive, so neighbouring workgroups also scan
  // similar tiles
  const int groups = (p.nq + MPW - 1) / MPW;
  const int gid = blockIdx.x * 4 + wv;
  const bool active = gid < NB3 * groups;
  const int s = active ? gid / groups : 0;
  const int i0 = active ? (gid - s * groups) * MPW : 0;
  double w[MPW];
  bool live_m[MPW];
  int qm[MPW];
#pragma unroll
  for (int k = 0; k < MPW; ++k) {
    const bool in = active && i0 + k < p.nq;
    const int q = in ? perm[(size_t)s * p.nq + i0 + k] : 0;
    qm[k] = q;
    const double2 r = in ? rec[(size_t)q * NB3 + s] : make_double2(__builtin_nan(""), 0.0);
    w[k] = r.x;
    live_m[k] = in && (r.x == r.x);
    if (in && lane < NB3) e0s[wv][k][lane] = etaT[((size_t)q * NB3 + s) * NB3 + lane];
  }
  __syncthreads();
  if (!active) return;
  double acc[MPW];
#pragma unroll
  for (int k = 0; k < MPW; ++k) acc[k] = 0.0;
  bool any_live = false;
#pragma unroll
  for (int k = 0; k < MPW; ++k) any_live |= live_m[k];
  if (any_live) {
    double wlo = INFINITY, whi = -INFINITY;
#pragma unroll
    for (int k = 0; k < MPW; ++k)
      if (live_m[k]) {
        wlo = fmin(wlo, w[k]);
        whi = fmax(whi, w[k]);
      }
    for (int s1 = 0; s1 < NB3; ++s1) {
      const double* rs = rng_lds + 3 * (size_t)s1 * p.nblk;
      // the tiles that can hold a partner within 2 sigma' of [wlo, whi] form
      // a run: the first has its highest w at least wlo - 2 sigma'_max of the
      // branch (binary search; the highest w rises with b over the non-empty
      // tiles, which come first), and the run ends at the first tile whose
      // lowest w lies past whi + 2 sigma'_max (lowest w never falls)
      // (the order follows the FP32 rounding of w: a tile's highest or lowest
      // w may exceed a later tile's by one FP32 ulp, 1.2e-7 w; both bounds
      // carry twice that)
      const double reach_max = 2.0 * rng_lds[3 * p.nblk * NB3 + s1] * (1.0 + 1e-12);
      const double t_lo = wlo - reach_max - 2.4e-7 * fabs(wlo);
      const double t_hi = whi + reach_max + 2.4e-7 * fabs(whi);
      int lo_b = 0, hi_b = p.nblk;
      while (lo_b < hi_b) {
        const int mid = (lo_b + hi_b) >> 1;
        const double h = rs[3 * mid + 1];
        // an empty tile (h = -inf) sits after every non-empty one: count it as high
        if (h >= t_lo || !(h > -INFINITY)) hi_b = mid;
        else lo_b = mid + 1;
      }
      for (int b = lo_b; b < p.nblk; ++b) {
        const double* r = rs + 3 * b;
        if (!(r[0] <= t_hi)) break;  // lowest w past reach (or an empty tile)
        const double reach = 2.0 * r[2] * (1.0 + 1e-12);
        // the tile can hold a partner with |w - w'| < 2 sigma' only if w lies
        // within reach of its range
        bool tile = false;
#pragma unroll
        for (int k = 0; k < MPW; ++k) tile |= live_m[k] && w[k] > r[0] - reach && w[k] < r[1] + reach;
        if (!tile) continue;
        for (int i1 = b * p.blk + lane; i1 < min(p.nq, (b + 1) * p.blk); i1 += 64) {
          const int q1 = perm[(size_t)s1 * p.nq + i1];
          const int m1 = q1 * NB3 + s1;
          const double2 o = rec[m1];
          bool pass[MPW];
          bool any = false;
#pragma unroll
          for (int k = 0; k < MPW; ++k) {
            pass[k] = live_m[k] && fabs(w[k] - o.x) < 2.0 * o.y;  // fails for partners below nu_min (NaN)
            any |= pass[k];
          }
          if (!any) continue;
          const double2 iv = inv[m1];
          double2 e1[NB3];
          const double2* e1p = etaT + (size_t)m1 * NB3;
#pragma unroll
          for (int j = 0; j < NB3; ++j) e1[j] = e1p[j];
#pragma unroll
          for (int k = 0; k < MPW; ++k) {
            if (!pass[k]) continue;
            double ov = 0.0;
#pragma unroll
            for (int i = 0; i < NB; ++i) {
              double dr = 0.0, di = 0.0;
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                const double2 u = e0s[wv][k][3 * i + a], v = e1[3 * i + a];
                // conj(u) v, as fused multiply-adds into the sums
                dr = fma(u.x, v.x, dr);
                dr = fma(u.y, v.y, dr);
                di = fma(u.x, v.y, di);
                di = fma(-u.y, v.x, di);
              }
              ov += p.g[i] * (dr * dr + di * di);
            }
            const double x = w[k] - o.x;
            double d;
            if (p.shape == KALDO_GAUSS) {
              const double u = x * iv.x;
              d = exp(-(u * u)) * iv.y;
            } else {
              d = smear(p.shape, x, o.y);
            }
            acc[k] += d * ov;
          }
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < MPW; ++k) {
    const double v = wave_sum_fixed(acc[k]);
    const int q = qm[k];
    if (lane == 0 && active && i0 + k < p.nq) {
      const size_t m = (size_t)q * NB3 + s;
      if (live_m[k]) {
        const double gi = p.scale * w[k] * w[k] * v;
        gamma[m] = accumulate ? gamma[m] + gi : gi;
      } else if (!accumulate) {
        gamma[m] = 0.0;  // below nu_min: no linewidth
      }
    }
  }
}

struct IsoWs {
  int blk, nblk;
  size_t off_rec, off_inv, off_eta, off_range, off_perm, total;
};

static IsoWs iso_ws(long nq, int nb3) {
  IsoWs w{};
  // tiles of 64 q-points, widened until the range table fits the LDS budget
  int blk = 64;
  while (((nq + blk - 1) / blk) * (size_t)nb3 * 3 * sizeof(double) > kIsoRangeLds) blk += 64;
  w.blk = blk;
  w.nblk = (int)((nq + blk - 1) / blk);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  w.off_rec = take(sizeof(double2) * nq * nb3);
  w.off_inv = take(sizeof(double2) * nq * nb3);
  w.off_eta = take(sizeof(double2) * nq * nb3 * nb3);
  w.off_range = take(sizeof(double) * (3 * (size_t)w.nblk * nb3 + nb3));
  w.off_perm = take(sizeof(int32_t) * (size_t)nq * nb3);
  w.total = o;
  return w;
}

}  // namespace kaldo

using namespace kaldo;

extern "C" size_t kaldo_isotope_workspace(const kaldo_crystal* c, const int32_t* mesh) {
  if (!c || !mesh || mesh[0] < 1 || mesh[1] < 1 || mesh[2] < 1) return 0;
  return iso_ws((long)mesh[0] * mesh[1] * mesh[2], c->nb3).total;
}

extern "C" int kaldo_isotope_linewidths(const kaldo_crystal* c, const int32_t* mesh,
                                        const double* omega, const double* evec,
                                        const double* vel, const double* g_factor,
                                        const kaldo_broadening* b, int32_t accumulate,
                                        void* workspace, size_t workspace_bytes, double* gamma,
                                        void* stream) {
  KALDO_REQUIRE(c && mesh && omega && evec && vel && g_factor && b && gamma,
                "kaldo_isotope_linewidths: NULL argument");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1,
                "kaldo_isotope_linewidths: mesh must be >= 1");
  KALDO_REQUIRE(c->nb <= kIsoMaxBasis, "kaldo_isotope_linewidths: more than 5 basis atoms");
  KALDO_REQUIRE(accumulate == 0 || accumulate == 1, "kaldo_isotope_linewidths: accumulate must be 0 or 1");
  int rc = check_broadening(b, true);
  if (rc) return rc;
  for (int i = 0; i < c->nb; ++i)
    KALDO_REQUIRE(std::isfinite(g_factor[i]) && g_factor[i] >= 0,
                  "kaldo_isotope_linewidths: g_factor must be finite and >= 0");
  const long nq = (long)mesh[0] * mesh[1] * mesh[2];
  KALDO_REQUIRE(nq <= 65535L, "kaldo_isotope_linewidths: mesh too large (N_q > 65535)");
  const IsoWs w = iso_ws(nq, c->nb3);
  KALDO_REQUIRE(workspace && workspace_bytes >= w.total,
                "kaldo_isotope_linewidths: workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  IsoParams p{};
  p.nq = (int)nq;
  p.nb3 = c->nb3;
  p.nb = c->nb;
  p.blk = w.blk;
  p.nblk = w.nblk;
  p.shape = b->shape;
  p.adaptive = b->adaptive;
  p.sig_fixed = kTwoPi * b->sigma_thz;
  p.sig_floor = kTwoPi * b->sigma_floor_thz;
  p.nu_min = b->nu_min_thz;
  p.scale = kPi / (2.0 * (double)nq);
  {
    double rc9[9];
    reciprocal(c->lattice, rc9);
    double h2 = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) {
        const double x = rc9[3 * r + k] / mesh[r];
        h2 += x * x;
      }
    p.h2 = h2 / 3.0;
  }
  for (int i = 0; i < c->nb; ++i) p.g[i] = g_factor[i];
  auto* ws = static_cast<unsigned char*>(workspace);
  auto* rec = reinterpret_cast<double2*>(ws + w.off_rec);
  auto* inv = reinterpret_cast<double2*>(ws + w.off_inv);
  auto* eta = reinterpret_cast<double2*>(ws + w.off_eta);
  auto* range = reinterpret_cast<double*>(ws + w.off_range);
  auto* perm = reinterpret_cast<int32_t*>(ws + w.off_perm);
  const int n_modes = (int)nq * c->nb3;
  KALDO_LAUNCH("iso_prep", iso_prep, dim3((n_modes + 255) / 256), dim3(256), 0, st, p, omega, vel,
               evec, rec, inv, eta, c->d_flags);
  // the frequency order of every branch, when its sort keys fit the LDS
  int dev = 0, lds_max = 0;
  KALDO_HIP(hipGetDevice(&dev));
  KALDO_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  size_t n2 = 1;
  while ((long)n2 < nq) n2 <<= 1;
  const int sorted = n2 * sizeof(unsigned long long) <= (size_t)lds_max ? 1 : 0;
  KALDO_LAUNCH("iso_sort", iso_sort, dim3(c->nb3), dim3(1024), sorted ? n2 * sizeof(unsigned long long) : 0,
               st, p, sorted, rec, perm);
  KALDO_LAUNCH("iso_ranges", iso_ranges, dim3((p.nblk * p.nb3 + 255) / 256), dim3(256), 0, st, p,
               perm, rec, range);
  KALDO_LAUNCH("iso_branch_smax", iso_branch_smax, dim3(1), dim3(64), 0, st, p, range);
  const size_t lds = sizeof(double) * (3 * (size_t)p.nblk * p.nb3 + p.nb3);
  const long n_waves = (long)c->nb3 * ((nq + kIsoMpw - 1) / kIsoMpw);
  const dim3 grid((unsigned)((n_waves + 3) / 4));
#define KALDO_ISO_CASE(NB3V)                                                                   \
  case NB3V:                                                                                   \
    KALDO_LAUNCH("iso_kernel", iso_kernel<NB3V>, grid, dim3(256), lds, st, p, rec, inv, eta, range, \
                 perm, accumulate, gamma);                                                     \
    break;
  switch (c->nb3) {
    KALDO_ISO_CASE(3)
    KALDO_ISO_CASE(6)
    KALDO_ISO_CASE(9)
    KALDO_ISO_CASE(12)
    KALDO_ISO_CASE(15)
    default:
      set_error("kaldo_isotope_linewidths: unsupported branch count");
      return KALDO_EUNSUPPORTED;
  }
#undef KALDO_ISO_CASE
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}
