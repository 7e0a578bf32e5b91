// Linewidths at many temperatures from the temperature cache.
//
// Paper: multi-temperature optimisation ("Performance and Scalability"):
// the projection of Eq. phi3_proj, and with it every factor of Eq. gamma
// but the populations, is computed once (kaldo_tcache_build); each
// temperature then costs one pass over the cached entries,
//   Gamma_mu(T) = pi hbar U^3/(8 N_q) sum_rows c (n1 - n2) + d (n1 + n2 + 1),
// with n = n_BE(w, T) of Eq. bose for the entry's two partner modes.
//
//   tc_occ     per mode: n(w, T_t) for a batch of NT temperatures, laid out
//              [mode][NT] so that one entry's populations at every T of the
//              batch are one contiguous gather per partner
//   tc_gamma   one wave per mode row: lanes stride over the row's entries
//              (coalesced 8-byte pair and 16-byte factor loads), gather the
//              two partners' populations, accumulate NT sums, and reduce
//              them across the wave in a fixed order (bitwise reproducible)
#include <algorithm>
#include <cmath>

#include "common.h"
#include "lw_common.h"

namespace kaldo {

constexpr int kTcMaxBatch = 8;

struct TcTemps {
  double inv_kt_hbar[kTcMaxBatch];  // hbar / (k_B T) per temperature of the batch
};

template <int NT>
__global__ void tc_occ(int n_modes, const double* __restrict__ omega, double nu_min, TcTemps t,
                       double* __restrict__ occ) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_modes) return;
  const double w = omega[m];
  const bool phys = (w / kTwoPi) >= nu_min;
#pragma unroll
  for (int k = 0; k < NT; ++k) occ[(size_t)m * NT + k] = phys ? 1.0 / expm1(w * t.inv_kt_hbar[k]) : 0.0;
}

template <int NT>
__global__ __launch_bounds__(256) void tc_gamma(int n_modes, const double* __restrict__ omega,
                                                double nu_min, const long long* __restrict__ row_ptr,
                                                long long n_entries, const uint2* __restrict__ pairs,
                                                const double2* __restrict__ factors,
                                                const double* __restrict__ occ, double scale,
                                                double* __restrict__ gamma, int32_t* flags) {
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= n_modes) return;
  long long lo = row_ptr[m], hi = row_ptr[m + 1];
  if (lo < 0 || hi < lo || hi > n_entries) {
    if (lane == 0) raise_flag(flags, kFlagCache);
    lo = hi = 0;
  }
  double acc[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) acc[k] = 0.0;
  for (long long e = lo + lane; e < hi; e += 64) {
    const uint2 ij = pairs[e];
    const double2 f = factors[e];
    if (ij.x >= (unsigned)n_modes || ij.y >= (unsigned)n_modes) {
      raise_flag(flags, kFlagCache);
      continue;
    }
    const double* n1 = occ + (size_t)ij.x * NT;
    const double* n2 = occ + (size_t)ij.y * NT;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const double a = n1[k], b = n2[k];
      acc[k] += f.x * (a - b) + f.y * ((a + b) + 1.0);
    }
  }
  const bool phys = (omega[m] / kTwoPi) >= nu_min;
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const double v = wave_sum_fixed(acc[k]);
    if (lane == 0) gamma[(size_t)k * n_modes + m] = phys ? scale * v : 0.0;
  }
}

template <int NT>
static void launch_batch(int n_modes, const double* omega, double nu_min, const TcTemps& t,
                         const long long* row_ptr, long long n_entries, const uint2* pairs,
                         const double2* factors, double* occ, double scale, double* gamma,
                         int32_t* flags, hipStream_t st) {
  KALDO_LAUNCH("tc_occ", tc_occ<NT>, dim3((n_modes + 255) / 256), dim3(256), 0, st, n_modes, omega,
               nu_min, t, occ);
  KALDO_LAUNCH("tc_gamma", tc_gamma<NT>, dim3((n_modes + 3) / 4), dim3(256), 0, st, n_modes, omega,
               nu_min, row_ptr, n_entries, pairs, factors, occ, scale, gamma, flags);
}

}  // namespace kaldo

using namespace kaldo;

extern "C" size_t kaldo_tcache_gamma_workspace(const kaldo_crystal* c, const int32_t* mesh) {
  if (!c || !mesh || mesh[0] < 1 || mesh[1] < 1 || mesh[2] < 1) return 0;
  const size_t n_modes = (size_t)mesh[0] * mesh[1] * mesh[2] * c->nb3;
  return n_modes * kTcMaxBatch * sizeof(double);
}

extern "C" int kaldo_tcache_gamma(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                                  double nu_min_thz, const int64_t* row_ptr, int64_t n_entries,
                                  const uint32_t* pairs, const double* factors, int32_t n_temps,
                                  const double* temperatures, void* workspace,
                                  size_t workspace_bytes, double* gamma, void* stream) {
  KALDO_REQUIRE(c && mesh && omega && row_ptr, "kaldo_tcache_gamma: NULL argument");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "kaldo_tcache_gamma: mesh must be >= 1");
  KALDO_REQUIRE(n_temps >= 0, "kaldo_tcache_gamma: n_temps < 0");
  KALDO_REQUIRE(n_entries >= 0, "kaldo_tcache_gamma: n_entries < 0");
  KALDO_REQUIRE(n_entries == 0 || (pairs && factors), "kaldo_tcache_gamma: NULL entries");
  KALDO_REQUIRE(std::isfinite(nu_min_thz) && nu_min_thz >= 0, "kaldo_tcache_gamma: nu_min_thz < 0");
  if (n_temps == 0) return KALDO_OK;
  KALDO_REQUIRE(temperatures && gamma, "kaldo_tcache_gamma: NULL temperatures or gamma");
  for (int k = 0; k < n_temps; ++k)
    KALDO_REQUIRE(std::isfinite(temperatures[k]) && temperatures[k] > 0,
                  "kaldo_tcache_gamma: temperatures must be finite and > 0");
  const long nq = (long)mesh[0] * mesh[1] * mesh[2];
  KALDO_REQUIRE(nq <= 65535L, "kaldo_tcache_gamma: mesh too large (N_q > 65535)");
  const int n_modes = (int)nq * c->nb3;
  KALDO_REQUIRE(workspace && workspace_bytes >= kaldo_tcache_gamma_workspace(c, mesh),
                "kaldo_tcache_gamma: workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* occ = static_cast<double*>(workspace);
  const double scale = kPrefactor / (double)nq;
  auto* rp = reinterpret_cast<const long long*>(row_ptr);
  auto* pr = reinterpret_cast<const uint2*>(pairs);
  auto* fa = reinterpret_cast<const double2*>(factors);
  // batches of 8, 4, 2 and 1 temperatures (largest first)
  for (int t0 = 0; t0 < n_temps;) {
    const int left = n_temps - t0;
    const int nt = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    TcTemps t{};
    for (int k = 0; k < nt; ++k) t.inv_kt_hbar[k] = kHbar / (kKb * temperatures[t0 + k]);
    double* g = gamma + (size_t)t0 * n_modes;
    switch (nt) {
      case 8:
        launch_batch<8>(n_modes, omega, nu_min_thz, t, rp, n_entries, pr, fa, occ, scale, g, c->d_flags, st);
        break;
      case 4:
        launch_batch<4>(n_modes, omega, nu_min_thz, t, rp, n_entries, pr, fa, occ, scale, g, c->d_flags, st);
        break;
      case 2:
        launch_batch<2>(n_modes, omega, nu_min_thz, t, rp, n_entries, pr, fa, occ, scale, g, c->d_flags, st);
        break;
      default:
        launch_batch<1>(n_modes, omega, nu_min_thz, t, rp, n_entries, pr, fa, occ, scale, g, c->d_flags, st);
    }
    t0 += nt;
  }
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}
