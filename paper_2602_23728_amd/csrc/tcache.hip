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
//   tc_gamma   one wave per mode row: entries loaded 64 per instruction,
//              handed to groups of NT/2 lanes of which each gathers two
//              temperatures of the two partners' populations, and a fixed
//              butterfly reduces the groups (bitwise reproducible)
#include <algorithm>
#include <cmath>
#include <cstdlib>

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

// One wave per mode row.  The row's entries are loaded 64 at a time, one
// per lane (contiguous 512-byte pair and 1 KiB factor reads), U such groups
// in flight, the next U issued before the current ones are used.  A
// partner's populations at the batch's NT temperatures are one 8 NT-byte row
// of the table; a lane gathers 16 bytes of it (two temperatures), so NT/2
// lanes work on one entry, taking its pair and factors from the lane that
// loaded it (cross-lane shuffles), and one gather instruction covers 128/NT
// entries.  Lanes holding the same temperatures are reduced by a fixed
// butterfly (bitwise reproducible).  A group past the row's end loads zero
// factors, which add exactly 0.
template <int NT>
__global__ __launch_bounds__(256) void tc_gamma(int n_modes, const double* __restrict__ omega,
                                                double nu_min, const long long* __restrict__ row_ptr,
                                                long long n_entries, const uint2* __restrict__ pairs,
                                                const double2* __restrict__ factors,
                                                const double* __restrict__ occ, double scale,
                                                double* __restrict__ gamma, int32_t* flags) {
  constexpr int TPL = NT >= 2 ? 2 : 1;  // temperatures per lane
  constexpr int LPE = NT / TPL;         // lanes per entry
  constexpr int EPW = 64 / LPE;         // entries per wave and gather
  constexpr int U = 4;                  // groups of 64 entries in flight
  const int lane = threadIdx.x & 63;
  const int sub = lane % LPE, grp = lane / LPE;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= n_modes) return;
  long long lo = row_ptr[m], hi = row_ptr[m + 1];
  if (lo < 0 || hi < lo || hi > n_entries) {
    if (lane == 0) raise_flag(flags, kFlagCache);
    lo = hi = 0;
  }
  double acc[TPL];
#pragma unroll
  for (int t = 0; t < TPL; ++t) acc[t] = 0.0;
  // one entry: its two partners' populations at this lane's temperatures (a
  // partner index out of range is skipped and reported)
  auto add = [&](uint2 ij, double2 f) {
    if (ij.x >= (unsigned)n_modes || ij.y >= (unsigned)n_modes) {
      raise_flag(flags, kFlagCache);
      return;
    }
    if constexpr (TPL == 2) {
      const double2 a = reinterpret_cast<const double2*>(occ + (size_t)ij.x * NT)[sub];
      const double2 b = reinterpret_cast<const double2*>(occ + (size_t)ij.y * NT)[sub];
      acc[0] += f.x * (a.x - b.x) + f.y * ((a.x + b.x) + 1.0);
      acc[1] += f.x * (a.y - b.y) + f.y * ((a.y + b.y) + 1.0);
    } else {
      const double a = occ[ij.x], b = occ[ij.y];
      acc[0] += f.x * (a - b) + f.y * ((a + b) + 1.0);
    }
  };
  auto load = [&](long long base, uint2* ij, double2* f) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long k = base + 64 * u + lane;
      if (k < hi) {
        // the entries stream through once per launch: non-temporal loads
        // leave the caches to the population rows the entries gather
        typedef unsigned nt_u2 __attribute__((ext_vector_type(2)));
        typedef double nt_d2 __attribute__((ext_vector_type(2)));
        const nt_u2 p2 = __builtin_nontemporal_load(reinterpret_cast<const nt_u2*>(pairs + k));
        const nt_d2 f2 = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(factors + k));
        ij[u] = make_uint2(p2.x, p2.y);
        f[u] = make_double2(f2.x, f2.y);
      } else {
        ij[u] = make_uint2(0u, 0u);
        f[u] = make_double2(0.0, 0.0);
      }
    }
  };
  constexpr long long BLK = 64LL * U;
  uint2 ij[U];
  double2 f[U];
  if (lo < hi) load(lo, ij, f);
  for (long long base = lo; base < hi; base += BLK) {
    uint2 cij[U];
    double2 cf[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cij[u] = ij[u];
      cf[u] = f[u];
    }
    if (base + BLK < hi) load(base + BLK, ij, f);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (LPE == 1) {
        add(cij[u], cf[u]);
      } else {
        // group grp takes entry 64 u + EPW j + grp, loaded by lane EPW j + grp
#pragma unroll
        for (int j = 0; j < LPE; ++j) {
          const int src = EPW * j + grp;
          uint2 e;
          e.x = (unsigned)__shfl((int)cij[u].x, src, 64);
          e.y = (unsigned)__shfl((int)cij[u].y, src, 64);
          double2 g;
          g.x = __shfl(cf[u].x, src, 64);
          g.y = __shfl(cf[u].y, src, 64);
          add(e, g);
        }
      }
    }
  }
  // lanes with the same `sub` hold the same temperatures
#pragma unroll
  for (int t = 0; t < TPL; ++t)
#pragma unroll
    for (int off = 32; off >= LPE; off >>= 1) acc[t] += __shfl_xor(acc[t], off, 64);
  const bool phys = (omega[m] / kTwoPi) >= nu_min;
  if (lane < LPE) {
#pragma unroll
    for (int t = 0; t < TPL; ++t)
      gamma[(size_t)(TPL * lane + t) * n_modes + m] = phys ? scale * acc[t] : 0.0;
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
  // batches of 8, 4, 2 and 1 temperatures (largest first; KALDO_TC_BATCH =
  // 1, 2, 4 or 8 caps the batch)
  int cap = kTcMaxBatch;
  if (const char* e = std::getenv("KALDO_TC_BATCH")) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2 || v == 4 || v == 8) cap = v;
  }
  for (int t0 = 0; t0 < n_temps;) {
    const int left = std::min(n_temps - t0, cap);
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
