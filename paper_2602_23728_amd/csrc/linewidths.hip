// Three-phonon linewidths of a crystal on a Gamma-centred mesh.
//
// Paper: Eq. phi3_proj (projection of Phi3 on three eigenvectors, here with
// the Bloch phases of Eq. dynmat_reciprocal and all-incoming momenta
// q + q1 + q2 = G), Eq. gamma with its Delta terms (populations paired as
// coalescence (n1 - n2) at w + w1 - w2 and decay 1/2 (n1 + n2 + 1) at
// w - w1 - w2), Eq. broadening (normalised Gaussian / Lorentzian, evaluated
// only where |x| < 2 sigma), Eq. bose.  Only partner pairs that pass the
// 2-sigma cut are projected ("Computational Implementation").
//
// Every path starts with
//   lw_prepare       per mode: populations, physical mask, subset flags and
//                    the FP32 (v, omega) copy the sweeps pre-classify with
// and then runs the fused kernel (lw_fused.hip), the dense MFMA kernel
// (lw_mfma.hip) or, when neither fits, the generic kernels below:
//   lw_round_evec    eta rounded to the contraction type
//   lw_atilde        per (q, e): A~_q[e][s] = sum_t coef_t eta_{i_t}(q,s)
//                    e^{+i q.R_{l''_t}}   (sparse COO x eta, first index)
//   lw_crystal       per (q, q1): FP64 cut and weights for every (s,s',s''),
//                    projection of the passing ones, wave-ordered partial sums
//   lw_finish        per mode: fixed-order sum of the partials, prefactor
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>

#include "common.h"
#include "lw_common.h"

namespace kaldo {

// modef[m] = (v, omega) in FP32 for the sweep's pre-classification, omega
// NaN below the frequency floor so that every comparison against the mode
// fails, as the physical mask demands.  Also validates the mode's inputs:
// a non-finite omega, v or eigenvector column raises kFlagNonFinite, an
// imaginary mode (omega < 0) with |nu| >= nu_min raises kFlagImaginary.
// mrec (when given): the FP64 record (w, n), (vx, vy), (vz, 0) the fused
// kernel reads per partner, three 16-byte loads instead of six scattered ones.
__global__ void lw_prepare(int n_modes, int nb3, const double* __restrict__ omega,
                           const double* __restrict__ vel, const double* __restrict__ evec,
                           double inv_kt_hbar, double nu_min, double* __restrict__ occ,
                           uint8_t* __restrict__ phys, uint8_t* __restrict__ sel,
                           float4* __restrict__ modef, double2* __restrict__ mrec, int sel_all,
                           int32_t* __restrict__ flags) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_modes) return;
  double w = omega[m];
  bool p = (w / kTwoPi) >= nu_min;
  phys[m] = p;
  occ[m] = p ? 1.0 / expm1(w * inv_kt_hbar) : 0.0;
  sel[m] = sel_all ? 1 : 0;
  const double v0 = vel[3 * (size_t)m], v1 = vel[3 * (size_t)m + 1], v2 = vel[3 * (size_t)m + 2];
  modef[m] = make_float4((float)v0, (float)v1, (float)v2, p ? (float)w : __builtin_nanf(""));
  if (mrec) {
    mrec[3 * (size_t)m] = make_double2(w, occ[m]);
    mrec[3 * (size_t)m + 1] = make_double2(v0, v1);
    mrec[3 * (size_t)m + 2] = make_double2(v2, 0.0);
  }
  // x - x is 0 for every finite x and NaN otherwise
  double chk = (w - w) + (v0 - v0) + (v1 - v1) + (v2 - v2);
  const int q = m / nb3, s = m - q * nb3;
  const double* col = evec + ((size_t)q * nb3 * nb3 + s) * 2;
  for (int j = 0; j < nb3; ++j) chk += (col[2 * j * nb3] - col[2 * j * nb3]) + (col[2 * j * nb3 + 1] - col[2 * j * nb3 + 1]);
  if (!(chk == 0.0)) raise_flag(flags, kFlagNonFinite);
  if (w < 0.0 && (-w / kTwoPi) >= nu_min) raise_flag(flags, kFlagImaginary);
}

__global__ void lw_select(const int32_t* __restrict__ subset, long n_subset, int n_modes,
                          uint8_t* __restrict__ sel, int32_t* __restrict__ flags) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_subset) return;
  int m = subset[k];
  if (m >= 0 && m < n_modes)
    sel[m] = 1;
  else
    raise_flag(flags, kFlagSubset);
}

template <typename T>
__global__ void lw_round_evec(long n, const double* __restrict__ evec, typename Cx<T>::type* out) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  out[k] = Cx<T>::make((T)evec[2 * k], (T)evec[2 * k + 1]);
}

// A~_q[e][s] for every q, e, s (complex in T, built in FP64).
template <typename T>
__global__ void lw_atilde(int nq, int nb3, int n_e, int N0, int N1, int N2,
                          const int32_t* __restrict__ rep, const int32_t* __restrict__ t_ptr,
                          const int32_t* __restrict__ t_i, const int32_t* __restrict__ t_l2,
                          const double* __restrict__ t_coef, const double* __restrict__ evec,
                          typename Cx<T>::type* __restrict__ at) {
  long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)nq * n_e * nb3;
  if (k >= total) return;
  int s = k % nb3;
  int e = (k / nb3) % n_e;
  int q = k / ((long)nb3 * n_e);
  int n0 = q / (N1 * N2), n1 = (q / N2) % N1, n2 = q % N2;
  double re = 0.0, im = 0.0;
  for (int t = t_ptr[e]; t < t_ptr[e + 1]; ++t) {
    const int32_t* r = rep + 3 * t_l2[t];
    int m0 = ((n0 * r[0]) % N0 + N0) % N0, m1 = ((n1 * r[1]) % N1 + N1) % N1,
        m2 = ((n2 * r[2]) % N2 + N2) % N2;
    double f = (double)m0 / N0 + (double)m1 / N1 + (double)m2 / N2;
    double sn, cs;
    sincospi(2.0 * f, &sn, &cs);  // e^{+i q.R''}
    size_t o = (((size_t)q * nb3 + t_i[t]) * nb3 + s) * 2;
    double ex = evec[o], ey = evec[o + 1];
    double c = t_coef[t];
    double px = c * (ex * cs - ey * sn), py = c * (ex * sn + ey * cs);
    re += px;
    im += py;
  }
  at[k] = Cx<T>::make((T)re, (T)im);
}

// One wave per (q, 64 consecutive q1); lane = q1.  Partial sums per
// (q, q1-block, s) in FP64, reduced across the wave in a fixed order.
template <typename T>
__global__ __launch_bounds__(64) void lw_crystal(LwParams p, const double* __restrict__ omega,
                                                 const double* __restrict__ vel,
                                                 const double* __restrict__ occ,
                                                 const uint8_t* __restrict__ phys,
                                                 const uint8_t* __restrict__ sel,
                                                 const typename Cx<T>::type* __restrict__ eta,
                                                 const typename Cx<T>::type* __restrict__ at,
                                                 const int32_t* __restrict__ dvec,
                                                 const int32_t* __restrict__ d_ptr,
                                                 const int32_t* __restrict__ e_jc,
                                                 const int32_t* __restrict__ e_kc,
                                                 double* __restrict__ partial) {
  using C = typename Cx<T>::type;
  extern __shared__ double2 smem_raw[];
  C* ph = reinterpret_cast<C*>(smem_raw);  // [n_d][64]
  const int lane = threadIdx.x;
  const int q = blockIdx.y;
  const int q1 = blockIdx.x * 64 + lane;
  const int nb3 = p.nb3;
  const bool valid = q1 < p.nq;
  const int N0 = p.N[0], N1 = p.N[1], N2 = p.N[2];
  const int a0 = q / (N1 * N2), a1 = (q / N2) % N1, a2 = q % N2;
  int q2 = 0;
  if (valid) {
    int b0 = q1 / (N1 * N2), b1 = (q1 / N2) % N1, b2 = q1 % N2;
    int c0 = ((-a0 - b0) % N0 + N0) % N0, c1 = ((-a1 - b1) % N1 + N1) % N1,
        c2 = ((-a2 - b2) % N2 + N2) % N2;
    q2 = (c0 * N1 + c1) * N2 + c2;
    // e^{-i q1.R_d}
    for (int d = 0; d < p.n_d; ++d) {
      const int32_t* r = dvec + 3 * d;
      int m0 = ((b0 * r[0]) % N0 + N0) % N0, m1 = ((b1 * r[1]) % N1 + N1) % N1,
          m2 = ((b2 * r[2]) % N2 + N2) % N2;
      double f = (double)m0 / N0 + (double)m1 / N1 + (double)m2 / N2;
      double sn, cs;
      sincospi(-2.0 * f, &sn, &cs);
      ph[d * 64 + lane] = Cx<T>::make((T)cs, (T)sn);
    }
  }
  __syncthreads();
  const C* eta1 = eta + (size_t)q1 * nb3 * nb3;
  const C* eta2 = eta + (size_t)q2 * nb3 * nb3;
  const C* atq = at + (size_t)q * p.n_e * nb3;
  for (int s = 0; s < nb3; ++s) {
    double acc = 0.0;
    const int mu = q * nb3 + s;
    if (valid && sel[mu] && phys[mu]) {
      const double w = omega[mu];
      for (int s1 = 0; s1 < nb3; ++s1) {
        const int m1 = q1 * nb3 + s1;
        if (!phys[m1]) continue;
        const double w1 = omega[m1], n1 = occ[m1];
        for (int s2 = 0; s2 < nb3; ++s2) {
          const int m2 = q2 * nb3 + s2;
          if (!phys[m2]) continue;
          const double w2 = omega[m2], n2 = occ[m2];
          double sp, sm;
          widths(p, vel, m1, m2, sp, sm);
          double wt = pair_weight(p, w, w1, w2, n1, n2, sp, sm);
          if (wt == 0.0) continue;
          // V = sum_d e^{-i q1.R_d} sum_{e in d} A~[e][s] eta1[jc][s1] eta2[kc][s2]
          T vr = 0, vi = 0;
          for (int d = 0; d < p.n_d; ++d) {
            T dr = 0, di = 0;
            for (int e = d_ptr[d]; e < d_ptr[d + 1]; ++e) {
              C a = atq[(size_t)e * nb3 + s];
              C x = eta1[e_jc[e] * nb3 + s1];
              C y = eta2[e_kc[e] * nb3 + s2];
              T xr = x.x * y.x - x.y * y.y, xi = x.x * y.y + x.y * y.x;
              dr += a.x * xr - a.y * xi;
              di += a.x * xi + a.y * xr;
            }
            C f = ph[d * 64 + lane];
            vr += f.x * dr - f.y * di;
            vi += f.x * di + f.y * dr;
          }
          double v2 = (double)vr * (double)vr + (double)vi * (double)vi;
          acc += v2 * wt;
        }
      }
    }
    acc = wave_sum_fixed(acc);
    if (lane == 0) partial[((size_t)q * gridDim.x + blockIdx.x) * nb3 + s] = acc;
  }
}

__global__ void lw_finish(int nq, int nb3, int nblk, double scale, const double* __restrict__ partial,
                          const uint8_t* __restrict__ phys, const uint8_t* __restrict__ sel,
                          double* __restrict__ gamma) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nq * nb3) return;
  if (!sel[m]) return;
  int q = m / nb3, s = m % nb3;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += partial[((size_t)q * nblk + b) * nb3 + s];
  gamma[m] = phys[m] ? scale * acc : 0.0;
}

// Which crystal kernel serves a request: the dense MFMA kernel for the split
// form (and, in FP32, for cells of 9 or more branches, where dense 16-wide
// tiles beat the pruned VALU path), otherwise the fused pruned kernel, and the
// generic kernel when neither fits.  KALDO_CRYSTAL_PATH=fused|mfma|generic
// overrides the FP32 choice.
enum class CrystalPath { Generic, Fused, Mfma };

static CrystalPath choose_path(const kaldo_crystal* c, int prec) {
  const char* env = std::getenv("KALDO_CRYSTAL_PATH");
  const std::string want = env ? env : "";
  if (prec == KALDO_BF16X3) {
    // The split form pays only on 16-wide matrix-core tiles; with fewer than
    // 9 branches they are mostly padding and the pruned FP32 kernel is much
    // faster (28x on the diamond 15^3 mesh) and at least as accurate, so
    // such requests run it (KALDO_CRYSTAL_PATH=mfma keeps the split form).
    if (want != "mfma" && c->nb3 < 9 && fused_supported(c, KALDO_FP32)) return CrystalPath::Fused;
    return CrystalPath::Mfma;
  }
  if (const char* f = std::getenv("KALDO_FORCE_GENERIC"))
    if (f[0] == '1') return CrystalPath::Generic;
  if (want == "generic") return CrystalPath::Generic;
  if (prec == KALDO_FP32 && mfma_supported(c) && (want == "mfma" || (want.empty() && c->nb3 >= 9)))
    return CrystalPath::Mfma;
  if (fused_supported(c, prec)) return CrystalPath::Fused;
  return CrystalPath::Generic;
}

// Workspace layout of the path that serves the request (offsets of buffers
// another path needs are left at 0 and never used).
struct CrystalWs {
  CrystalPath path;
  size_t off_occ, off_phys, off_sel, off_eta, off_at, off_partial, off_phase, off_modef, off_qlist,
      off_fpart, off_mrec, total;
};

static CrystalWs crystal_ws_for(const kaldo_crystal* c, long nq, int prec, CrystalPath path) {
  const int nb3 = c->nb3;
  const size_t cs = prec == KALDO_FP64 ? 16 : 8;
  const long nblk = (nq + 63) / 64;
  CrystalWs w{};
  w.path = path;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  w.off_occ = take(sizeof(double) * nq * nb3);
  w.off_phys = take(nq * nb3);
  w.off_sel = take(nq * nb3);
  w.off_modef = take(sizeof(float4) * nq * nb3);
  if (w.path == CrystalPath::Generic) {
    w.off_eta = take(cs * nq * nb3 * nb3);
    w.off_at = take(cs * nq * (size_t)c->bloch.n_e * nb3);
    w.off_partial = take(sizeof(double) * nq * nblk * nb3);
  } else if (w.path == CrystalPath::Fused) {
    w.off_eta = take(cs * nq * nb3 * nb3);
    w.off_phase = take(cs * nq * (size_t)std::max(1, c->bloch.n_d));
    w.off_qlist = take(sizeof(int32_t) * (2 * nq + 1));
    w.off_fpart = take(sizeof(double) * nq * kFusedMaxChunks * nb3);
    w.off_mrec = take(sizeof(double2) * 3 * nq * nb3);
  } else {
    w.off_phase = take(sizeof(float2) * nq * (size_t)std::max(1, c->bloch.n_d));
  }
  w.total = o;
  return w;
}

static CrystalWs crystal_ws(const kaldo_crystal* c, long nq, int prec) {
  return crystal_ws_for(c, nq, prec, choose_path(c, prec));
}

template <typename T>
static int run_crystal(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                       const double* evec, const double* vel, double T_k,
                       const kaldo_broadening* b, const int32_t* subset, int64_t n_subset,
                       unsigned char* ws, const CrystalWs& w, int prec, double* gamma,
                       hipStream_t st) {
  using C = typename Cx<T>::type;
  const int nb3 = c->nb3;
  const long nq = (long)mesh[0] * mesh[1] * mesh[2];
  const int n_modes = nq * nb3;
  double* occ = reinterpret_cast<double*>(ws + w.off_occ);
  uint8_t* phys = ws + w.off_phys;
  uint8_t* sel = ws + w.off_sel;
  C* eta = reinterpret_cast<C*>(ws + w.off_eta);
  C* at = reinterpret_cast<C*>(ws + w.off_at);
  double* partial = reinterpret_cast<double*>(ws + w.off_partial);
  float4* modef = reinterpret_cast<float4*>(ws + w.off_modef);
  double2* mrec = w.path == CrystalPath::Fused ? reinterpret_cast<double2*>(ws + w.off_mrec) : nullptr;
  const double inv_kt_hbar = kHbar / (kKb * T_k);
  KALDO_LAUNCH("lw_prepare", lw_prepare, dim3((n_modes + 255) / 256), dim3(256), 0, st, n_modes,
               nb3, omega, vel, evec, inv_kt_hbar, b->nu_min_thz, occ, phys, sel, modef, mrec,
               subset ? 0 : 1, c->d_flags);
  if (subset && n_subset > 0)
    KALDO_LAUNCH("lw_select", lw_select, dim3((n_subset + 255) / 256), dim3(256), 0, st, subset,
                 (long)n_subset, n_modes, sel, c->d_flags);
  LwParams p = make_params(c, mesh, T_k, b);
  const CrystalPath path = w.path;
  if (path == CrystalPath::Mfma) {
    float2* phase_tab = reinterpret_cast<float2*>(ws + w.off_phase);
    return launch_mfma(c, p, prec == KALDO_BF16X3, omega, vel, occ, phys, sel, evec, phase_tab,
                       kPrefactor / (double)nq, gamma, st);
  }
  if (path == CrystalPath::Fused) {
    C* phase_tab = reinterpret_cast<C*>(ws + w.off_phase);
    int32_t* qlist = reinterpret_cast<int32_t*>(ws + w.off_qlist);
    double* fpart = reinterpret_cast<double*>(ws + w.off_fpart);
    return launch_fused<T>(c, p, omega, vel, modef, occ, mrec, phys, sel, evec, eta, phase_tab, qlist,
                           fpart, subset ? n_subset : 0, kPrefactor / (double)nq, gamma, st);
  }
  long ne = nq * nb3 * nb3;
  KALDO_LAUNCH("lw_round_evec", lw_round_evec<T>, dim3((ne + 255) / 256), dim3(256), 0, st, ne, evec, eta);
  long na = nq * (long)c->bloch.n_e * nb3;
  KALDO_LAUNCH("lw_atilde", lw_atilde<T>, dim3((na + 255) / 256), dim3(256), 0, st, (int)nq, nb3,
                     c->bloch.n_e, mesh[0], mesh[1], mesh[2], c->d_rep, c->bloch.t_ptr,
                     c->bloch.t_i, c->bloch.t_l2, c->bloch.t_coef, evec, at);
  const int nblk = (nq + 63) / 64;
  size_t shmem = sizeof(C) * 64 * std::max(1, c->bloch.n_d);
  KALDO_LAUNCH("lw_crystal", lw_crystal<T>, dim3(nblk, nq), dim3(64), shmem, st, p, omega, vel, occ, phys,
                     sel, eta, at, c->bloch.dvec, c->bloch.d_ptr, c->bloch.e_jc, c->bloch.e_kc,
                     partial);
  KALDO_LAUNCH("lw_finish", lw_finish, dim3((n_modes + 255) / 256), dim3(256), 0, st, (int)nq, nb3, nblk,
                     kPrefactor / (double)nq, partial, phys, sel, gamma);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

}  // namespace kaldo

using namespace kaldo;

extern "C" size_t kaldo_linewidths_workspace(const kaldo_crystal* c, const int32_t* mesh,
                                             int32_t precision) {
  if (!c || !mesh || mesh[0] < 1 || mesh[1] < 1 || mesh[2] < 1) return 0;
  return crystal_ws(c, (long)mesh[0] * mesh[1] * mesh[2], precision).total;
}

namespace kaldo {

// Validation and enqueue of kaldo_linewidths on a given workspace (shared by
// the entry points that differ only in where the workspace comes from).
int linewidths_enqueue(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                       const double* evec, const double* vel, double temperature,
                       const kaldo_broadening* b, int32_t precision,
                       const int32_t* modes_subset, int64_t n_subset, void* workspace,
                       size_t workspace_bytes, double* gamma, hipStream_t st) {
  KALDO_REQUIRE(c && mesh && omega && evec && vel && b && gamma, "kaldo_linewidths: NULL argument");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "kaldo_linewidths: mesh must be >= 1");
  KALDO_REQUIRE(c->nb3 <= kMaxNb3Linewidths, "kaldo_linewidths: nb3 > 16 (use kaldo_linewidths_gamma)");
  KALDO_REQUIRE(std::isfinite(temperature) && temperature > 0, "kaldo_linewidths: temperature <= 0");
  int rc = check_broadening(b, true);
  if (rc) return rc;
  KALDO_REQUIRE(precision == KALDO_FP64 || precision == KALDO_FP32 || precision == KALDO_BF16X3,
                "kaldo_linewidths: unknown precision");
  if (precision == KALDO_BF16X3 && choose_path(c, precision) == CrystalPath::Mfma &&
      !mfma_supported(c)) {
    set_error("kaldo_linewidths: BF16X3 needs the MFMA kernel (nb3 <= 16, tables in LDS)");
    return KALDO_EUNSUPPORTED;
  }
  KALDO_REQUIRE(n_subset >= 0 && (n_subset == 0 || modes_subset), "kaldo_linewidths: bad subset");
  const long nq = (long)mesh[0] * mesh[1] * mesh[2];
  KALDO_REQUIRE(nq <= 65535L, "kaldo_linewidths: mesh too large (N_q > 65535)");
  CrystalWs w = crystal_ws(c, nq, precision);
  KALDO_REQUIRE(workspace && workspace_bytes >= w.total, "kaldo_linewidths: workspace too small");
  if (modes_subset && n_subset == 0) return KALDO_OK;
  auto* ws = static_cast<unsigned char*>(workspace);
  if (precision == KALDO_FP64)
    return run_crystal<double>(c, mesh, omega, evec, vel, temperature, b, modes_subset, n_subset,
                               ws, w, precision, gamma, st);
  return run_crystal<float>(c, mesh, omega, evec, vel, temperature, b, modes_subset, n_subset, ws,
                            w, precision, gamma, st);
}

}  // namespace kaldo

extern "C" int kaldo_linewidths(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                                const double* evec, const double* vel, double temperature,
                                const kaldo_broadening* b, int32_t precision,
                                const int32_t* modes_subset, int64_t n_subset, void* workspace,
                                size_t workspace_bytes, double* gamma, void* stream) {
  return linewidths_enqueue(c, mesh, omega, evec, vel, temperature, b, precision, modes_subset,
                            n_subset, workspace, workspace_bytes, gamma,
                            static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// Temperature cache: the temperature-independent factors of Eq. gamma for
// every cut-passing partner entry, built by the fused kernel's count and
// record passes (the sweeps over temperature are in tcache.hip).

using namespace kaldo;

extern "C" size_t kaldo_tcache_workspace(const kaldo_crystal* c, const int32_t* mesh,
                                         int32_t precision) {
  if (!c || !mesh || mesh[0] < 1 || mesh[1] < 1 || mesh[2] < 1) return 0;
  return crystal_ws_for(c, (long)mesh[0] * mesh[1] * mesh[2], precision, CrystalPath::Fused).total;
}

extern "C" int kaldo_tcache_build(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                                  const double* evec, const double* vel,
                                  const kaldo_broadening* b, int32_t precision,
                                  const int32_t* modes_subset, int64_t n_subset, void* workspace,
                                  size_t workspace_bytes, int64_t* row_ptr, int64_t capacity,
                                  uint32_t* pairs, double* factors, int64_t* n_entries,
                                  void* stream) {
  KALDO_REQUIRE(c && mesh && omega && evec && vel && b && row_ptr && n_entries,
                "kaldo_tcache_build: NULL argument");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "kaldo_tcache_build: mesh must be >= 1");
  KALDO_REQUIRE(c->nb3 <= kMaxNb3Linewidths, "kaldo_tcache_build: nb3 > 16");
  int rc = check_broadening(b, true);
  if (rc) return rc;
  KALDO_REQUIRE(precision == KALDO_FP64 || precision == KALDO_FP32 || precision == KALDO_BF16X3,
                "kaldo_tcache_build: unknown precision");
  if (precision == KALDO_BF16X3 || !fused_record_supported(c, precision)) {
    set_error("kaldo_tcache_build: needs the fused kernel (FP64 or FP32, at most 5 basis atoms, "
              "64 replicas, A~ tables and record queue in LDS)");
    return KALDO_EUNSUPPORTED;
  }
  KALDO_REQUIRE(n_subset >= 0 && (n_subset == 0 || modes_subset), "kaldo_tcache_build: bad subset");
  KALDO_REQUIRE(capacity >= 0, "kaldo_tcache_build: capacity < 0");
  KALDO_REQUIRE((pairs == nullptr) == (factors == nullptr),
                "kaldo_tcache_build: pairs and factors must both be given or both be NULL");
  const long nq = (long)mesh[0] * mesh[1] * mesh[2];
  KALDO_REQUIRE(nq <= 65535L, "kaldo_tcache_build: mesh too large (N_q > 65535)");
  const CrystalWs w = crystal_ws_for(c, nq, precision, CrystalPath::Fused);
  KALDO_REQUIRE(workspace && workspace_bytes >= w.total, "kaldo_tcache_build: workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nb3 = c->nb3;
  const int n_modes = (int)nq * nb3;
  *n_entries = 0;
  if (modes_subset && n_subset == 0) {
    KALDO_HIP(hipMemsetAsync(row_ptr, 0, sizeof(int64_t) * (n_modes + 1), st));
    KALDO_HIP(hipStreamSynchronize(st));
    return KALDO_OK;
  }
  auto* ws = static_cast<unsigned char*>(workspace);
  double* occ = reinterpret_cast<double*>(ws + w.off_occ);
  uint8_t* phys = ws + w.off_phys;
  uint8_t* sel = ws + w.off_sel;
  float4* modef = reinterpret_cast<float4*>(ws + w.off_modef);
  double2* mrec = reinterpret_cast<double2*>(ws + w.off_mrec);
  int32_t* qlist = reinterpret_cast<int32_t*>(ws + w.off_qlist);
  // the populations lw_prepare writes are not used: any temperature will do
  KALDO_LAUNCH("lw_prepare", lw_prepare, dim3((n_modes + 255) / 256), dim3(256), 0, st, n_modes, nb3,
               omega, vel, evec, kHbar / (kKb * 300.0), b->nu_min_thz, occ, phys, sel, modef, mrec,
               modes_subset ? 0 : 1, c->d_flags);
  if (modes_subset)
    KALDO_LAUNCH("lw_select", lw_select, dim3((n_subset + 255) / 256), dim3(256), 0, st,
                 modes_subset, (long)n_subset, n_modes, sel, c->d_flags);
  const LwParams p = make_params(c, mesh, 300.0, b);
  TcOut tc{reinterpret_cast<long long*>(ws + w.off_fpart), reinterpret_cast<long long*>(row_ptr),
           reinterpret_cast<uint2*>(pairs), reinterpret_cast<double2*>(factors), c->d_flags};
  const int64_t ns = modes_subset ? n_subset : 0;
  auto pass = [&](int mode) {
    if (precision == KALDO_FP64)
      return launch_fused_cache<double>(c, p, mode, omega, vel, modef, mrec, phys, sel, evec,
                                        reinterpret_cast<double2*>(ws + w.off_eta),
                                        reinterpret_cast<double2*>(ws + w.off_phase), qlist, ns, tc, st);
    return launch_fused_cache<float>(c, p, mode, omega, vel, modef, mrec, phys, sel, evec,
                                     reinterpret_cast<float2*>(ws + w.off_eta),
                                     reinterpret_cast<float2*>(ws + w.off_phase), qlist, ns, tc, st);
  };
  rc = pass(kModeCount);
  if (rc) return rc;
  int64_t total = 0;
  KALDO_HIP(hipMemcpyAsync(&total, row_ptr + n_modes, sizeof(total), hipMemcpyDeviceToHost, st));
  KALDO_HIP(hipStreamSynchronize(st));
  *n_entries = total;
  if (!pairs) return KALDO_OK;
  if (capacity < total) {
    set_error("kaldo_tcache_build: capacity " + std::to_string(capacity) + " below the " +
              std::to_string(total) + " entries needed");
    return KALDO_EINVAL;
  }
  return pass(kModeRecord);
}
