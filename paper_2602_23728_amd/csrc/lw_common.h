// Device helpers shared by the crystal and Gamma-point linewidth kernels:
// the FP64 energy cut, smearing and population weight of one partner pair,
// adaptive widths, and a fixed-order wave reduction.
#pragma once

#include <cmath>

#include "common.h"

namespace kaldo {

// pi hbar U^3 / 8: turns sum |V|^2 [eV^2/(A^6 amu^3)] w^-3 g [ps^4] into rad/ps.
constexpr double kPrefactor = kPi * kHbar * kU * kU * kU / 8.0;

template <typename T>
struct Cx;
template <>
struct Cx<float> {
  using type = float2;
  __host__ __device__ static float2 make(float x, float y) { return make_float2(x, y); }
};
template <>
struct Cx<double> {
  using type = double2;
  __host__ __device__ static double2 make(double x, double y) { return make_double2(x, y); }
};

struct LwParams {
  int nb3, nq, n_d, n_e, n_blk;
  int N[3];
  int shape, adaptive;
  int half;  // Phi3 symmetric in its last two slots: mirrored partner pairs share V
  double sig_fixed, sig_floor, h2;  // rad/ps, rad/ps, 1/A^2
};

inline int check_broadening(const kaldo_broadening* b, bool allow_adaptive) {
  KALDO_REQUIRE(b->shape == KALDO_GAUSS || b->shape == KALDO_LORENTZ, "broadening: unknown shape");
  KALDO_REQUIRE(b->adaptive == 0 || b->adaptive == 1, "broadening: adaptive must be 0 or 1");
  KALDO_REQUIRE(allow_adaptive || b->adaptive == 0,
                "broadening: adaptive widths need group velocities (crystal path only)");
  if (b->adaptive)
    KALDO_REQUIRE(std::isfinite(b->sigma_floor_thz) && b->sigma_floor_thz > 0,
                  "broadening: sigma_floor_thz must be > 0");
  else
    KALDO_REQUIRE(std::isfinite(b->sigma_thz) && b->sigma_thz > 0, "broadening: sigma_thz must be > 0");
  KALDO_REQUIRE(std::isfinite(b->nu_min_thz) && b->nu_min_thz >= 0, "broadening: nu_min_thz < 0");
  return KALDO_OK;
}

inline LwParams make_params(const kaldo_crystal* c, const int32_t* mesh, double T,
                            const kaldo_broadening* b) {
  LwParams p;
  p.nb3 = c->nb3;
  p.nq = mesh[0] * mesh[1] * mesh[2];
  p.n_d = c->bloch.n_d;
  p.n_e = c->bloch.n_e;
  p.n_blk = c->bloch.n_blk;
  p.half = c->bloch.sym_jk;
  for (int i = 0; i < 3; ++i) p.N[i] = mesh[i];
  p.shape = b->shape;
  p.adaptive = b->adaptive;
  p.sig_fixed = kTwoPi * b->sigma_thz;
  p.sig_floor = kTwoPi * b->sigma_floor_thz;
  double rc[9];
  reciprocal(c->lattice, rc);
  double h2 = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      double x = rc[3 * r + k] / mesh[r];
      h2 += x * x;
    }
  p.h2 = h2 / 3.0;
  (void)T;
  return p;
}

// sigma+ for coalescence (dv = v1 + v2), sigma- for decay (dv = -v1 + v2).
__device__ __forceinline__ void widths_v(const LwParams& p, const double* v1, const double* v2,
                                         double& sp, double& sm);
__device__ __forceinline__ void widths(const LwParams& p, const double* __restrict__ vel, int m1,
                                       int m2, double& sp, double& sm) {
  widths_v(p, vel + 3 * (size_t)m1, vel + 3 * (size_t)m2, sp, sm);
}
__device__ __forceinline__ void widths_v(const LwParams& p, const double* v1, const double* v2,
                                         double& sp, double& sm) {
  if (!p.adaptive) {
    sp = sm = p.sig_fixed;
    return;
  }
  double ax = v1[0] + v2[0], ay = v1[1] + v2[1], az = v1[2] + v2[2];
  double bx = -v1[0] + v2[0], by = -v1[1] + v2[1], bz = -v1[2] + v2[2];
  double Sa = ax * ax + ay * ay + az * az;
  double Sb = bx * bx + by * by + bz * bz;
  sp = fmax(sqrt(Sa * p.h2 / 12.0), p.sig_floor);
  sm = fmax(sqrt(Sb * p.h2 / 12.0), p.sig_floor);
}

// sigma^2 (not sigma) of the two processes, max(S h^2 / 12, floor^2), and
// the squared velocity sums S+- they come from (fixed width: S = 0).
__device__ __forceinline__ void widths2(const LwParams& p, const double* v1, const double* v2,
                                        double& s2p, double& s2m, double& Sp, double& Sm) {
  // no fused multiply-adds: the cut decisions made from S must come out the
  // same in every kernel that takes them (the cache's count and record
  // passes place entries by them), in the order the sums are written
#pragma clang fp contract(off)
  if (!p.adaptive) {
    s2p = s2m = p.sig_fixed * p.sig_fixed;
    Sp = Sm = 0.0;
    return;
  }
  const double ax = v1[0] + v2[0], ay = v1[1] + v2[1], az = v1[2] + v2[2];
  const double bx = -v1[0] + v2[0], by = -v1[1] + v2[1], bz = -v1[2] + v2[2];
  Sp = ax * ax + ay * ay + az * az;
  Sm = bx * bx + by * by + bz * bz;
  const double f2 = p.sig_floor * p.sig_floor;
  s2p = fmax(Sp * p.h2 / 12.0, f2);
  s2m = fmax(Sm * p.h2 / 12.0, f2);
}

__device__ __forceinline__ double smear(int shape, double x, double s) {
  if (shape == KALDO_GAUSS) return exp(-(x * x) / (s * s)) / (kSqrtPi * s);
  return (0.5 * s) / (kPi * (x * x + 0.25 * s * s));
}

// [(n1 - n2) g(x+) + 1/2 (n1 + n2 + 1) g(x-)] / (w w1 w2), zero unless a
// process passes |x| < 2 sigma; x+ = (w + w1) - w2, x- = (w - w1) - w2.
__device__ __forceinline__ double pair_weight(const LwParams& p, double w, double w1, double w2,
                                              double n1, double n2, double sp, double sm) {
  const double xp = (w + w1) - w2;
  const double xm = (w - w1) - w2;
  const bool pp = fabs(xp) < 2.0 * sp;
  const bool pm = fabs(xm) < 2.0 * sm;
  if (!(pp || pm)) return 0.0;
  if (p.shape == KALDO_GAUSS) {
    // the same value with two divisions instead of five: one reciprocal of
    // sigma+ sigma- gives both 1/sigma, and 1/(sqrt(pi) w w1 w2) is applied
    // once (the cut decisions above keep their exact form)
    const double r = 1.0 / (sp * sm);
    const double ip = sm * r, im = sp * r;
    double gp = 0.0, gm = 0.0;
    if (pp) {
      const double u = xp * ip;
      gp = exp(-(u * u)) * ip;
    }
    if (pm) {
      const double u = xm * im;
      gm = exp(-(u * u)) * im;
    }
    return ((n1 - n2) * gp + 0.5 * (n1 + n2 + 1.0) * gm) / (kSqrtPi * (w * (w1 * w2)));
  }
  const double gp = pp ? smear(p.shape, xp, sp) : 0.0;
  const double gm = pm ? smear(p.shape, xm, sm) : 0.0;
  const double pop = (n1 - n2) * gp + 0.5 * (n1 + n2 + 1.0) * gm;
  return pop / (w * (w1 * w2));
}

// The temperature-independent factors of one ordered partner pair:
// ap = g(x+; sigma+)/(w w1 w2) and am = g(x-; sigma-)/(w w1 w2), each zero
// unless its own process passes |x| < 2 sigma (the cut of pair_weight).
__device__ __forceinline__ void pair_factors(const LwParams& p, double w, double w1, double w2,
                                             double sp, double sm, double& ap, double& am) {
  const double xp = (w + w1) - w2;
  const double xm = (w - w1) - w2;
  const double den = w * (w1 * w2);
  ap = fabs(xp) < 2.0 * sp ? smear(p.shape, xp, sp) / den : 0.0;
  am = fabs(xm) < 2.0 * sm ? smear(p.shape, xm, sm) / den : 0.0;
}

// FP32 pre-classification of |x| < T against an FP64 reference: a_f is |x|
// evaluated in FP32 from FP32-rounded frequencies, whose error is bounded by
// 2u(|w| + |w1| + |w2|) (u = 2^-24); T_f = 2 sqrt(sigma^2) in FP32 is within
// a few ulp of 2 sigma.  Candidates outside [lo, hi] are decided here with
// certainty; the rest get the exact FP64 test.
struct Band {
  float lo, hi;
};

// The hardware square root (v_sqrt_f32, within 1 ulp for the normal inputs
// the bands see: sigma^2 >= floor^2), without the correctly-rounded
// expansion the compiler emits for sqrtf.  The bands carry a 1e-6 relative
// margin (about 17 ulp), so the pre-classification stays conservative.
__device__ __forceinline__ float band_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// The band [lo, hi] around T = 2 sigma for widths computed from the FP32
// mode copy (see widths2_f): d covers the FP32 error of |x| (scale_sum =
// |w| + |w1| + |w2|), e_sig how far 2 sigma computed that way can lie from
// 2 sigma computed in FP64, and the 1e-6 relative margin the rounding of T.
__device__ __forceinline__ Band make_band_f(float sig2, float scale_sum, float e_sig) {
  const float t = 2.0f * band_sqrt(sig2);
  const float d = 4e-7f * scale_sum + 1e-9f + e_sig;
  return {t * (1.0f - 1e-6f) - d, t * (1.0f + 1e-6f) + d};
}

// sigma^2 of both processes from FP32 velocities, and e_sig >= |2 sigma_f -
// 2 sigma| against sigma from the FP64 velocities.  With u = 2^-24, each
// component of v1 +- v2 is off by at most 2u (|v1_i| + |v2_i|), so
// |S_f - S| <= 7.001 u (S+ + S-), using sum_i (|v1_i| + |v2_i|)^2 <=
// 2 (|v1|^2 + |v2|^2) = S+ + S-; max(., floor^2) is 1-Lipschitz and
// |sqrt x - sqrt y| <= sqrt|x - y|, hence |2 sigma_f - 2 sigma| <=
// 2 sqrt(7.001 u (S+ + S-) h^2/12).  e_sig takes twice that; relative
// rounding of the constants and products is left to make_band_f's 1e-6.
__device__ __forceinline__ void widths2_f(const LwParams& p, float4 v1, float4 v2, float& s2p,
                                          float& s2m, float& e_sig) {
  if (!p.adaptive) {
    s2p = s2m = (float)(p.sig_fixed * p.sig_fixed);
    e_sig = 0.0f;
    return;
  }
  const float ax = v1.x + v2.x, ay = v1.y + v2.y, az = v1.z + v2.z;
  const float bx = v2.x - v1.x, by = v2.y - v1.y, bz = v2.z - v1.z;
  const float Sp = ax * ax + ay * ay + az * az, Sm = bx * bx + by * by + bz * bz;
  const float H = (float)(p.h2 / 12.0), F = (float)(p.sig_floor * p.sig_floor);
  s2p = fmaxf(Sp * H, F);
  s2m = fmaxf(Sm * H, F);
  e_sig = 2.0f * band_sqrt(1.7e-6f * (Sp + Sm) * H);
}

// The exact FP64 decision of the oracle: |(w + w1) - w2| < 2 sigma+ or
// |(w - w1) - w2| < 2 sigma-, sigma = max(sqrt(S h^2/12), floor) (or fixed).
__device__ __forceinline__ bool exact_pass(const LwParams& p, double w, double w1, double w2,
                                        double Sp, double Sm, bool plus) {
  double s;
  if (!p.adaptive)
    s = p.sig_fixed;
  else
    s = fmax(sqrt((plus ? Sp : Sm) * p.h2 / 12.0), p.sig_floor);
  const double x = plus ? (w + w1) - w2 : (w - w1) - w2;
  return fabs(x) < 2.0 * s;
}

// Sum over a wave64 in a fixed butterfly order; lane 0 holds the result.
__device__ __forceinline__ double wave_sum_fixed(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// e^{-i q1.R_d} for every mesh point q1 and replica difference d, in T.
template <typename T>
__global__ void lw_phase_table(int nq, int n_d, int N0, int N1, int N2,
                               const int32_t* __restrict__ dvec, typename Cx<T>::type* out) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long)nq * n_d) return;
  const int q1 = k / n_d, d = k % n_d;
  const int b0 = q1 / (N1 * N2), b1 = (q1 / N2) % N1, b2 = q1 % N2;
  const int32_t* r = dvec + 3 * d;
  int m0 = ((b0 * r[0]) % N0 + N0) % N0, m1 = ((b1 * r[1]) % N1 + N1) % N1,
      m2 = ((b2 * r[2]) % N2 + N2) % N2;
  double f = (double)m0 / N0 + (double)m1 / N1 + (double)m2 / N2;
  double sn, cs;
  sincospi(-2.0 * f, &sn, &cs);
  out[k] = Cx<T>::make((T)cs, (T)sn);
}

// Partner coordinates of one mesh dimension for a q with coordinate a: with
// t = (-a) mod N the partner of b is c(b) = (t - b) mod N, and b < c(b)
// exactly for b in [0, ceil(t/2)) and [t + 1, ceil((t + N)/2)) ("L", nL
// values), b == c(b) for b = t/2 (t even) and b = (t + N)/2 (t + N even)
// ("E", nE values).
// (t - b) mod N for t, b in [0, N): with t = (-a) mod N this is the
// coordinate of q2 = -q - q1 on the mesh, without an integer division.
__device__ __forceinline__ int wrap_sub(int t, int b, int N) {
  const int c = t - b;
  return c < 0 ? c + N : c;
}

struct HalfDim {
  int t, len1, nL, nE, e0, e1;
  __device__ int L(int j) const { return j < len1 ? j : t + 1 + (j - len1); }
  __device__ int E(int j) const { return j == 0 ? e0 : e1; }
};
__device__ inline HalfDim half_dim(int a, int N) {
  HalfDim h;
  h.t = (N - a) % N;
  h.len1 = (h.t + 1) / 2;
  h.nL = h.len1 + (h.t + N + 1) / 2 - h.t - 1;
  h.nE = 0;
  h.e0 = h.e1 = 0;
  if ((h.t & 1) == 0) h.e0 = h.t / 2, h.nE = 1;
  if (((h.t + N) & 1) == 0) {
    if (h.nE == 0)
      h.e0 = (h.t + N) / 2;
    else
      h.e1 = (h.t + N) / 2;
    ++h.nE;
  }
  return h;
}

// The swept partners q1 of one q in a fixed order.  Symmetric Phi3: the mesh
// points with q1 <_lex q2 (coordinates compared lexicographically, which is
// the flat order) in three ranges -- b0 in L0; b0 in E0, b1 in L1; b0 in E0,
// b1 in E1, b2 in L2 -- each doubled, then the points with q1 == q2 (E0 x E1
// x E2) once.  Otherwise every q1 once, in flat order.
struct Partners {
  HalfDim h[3];
  int nA, nB, nC, n;
  bool half;
  __device__ Partners(bool half_, int a0, int a1, int a2, int N0, int N1, int N2) : half(half_) {
    h[0] = half_dim(a0, N0);
    h[1] = half_dim(a1, N1);
    h[2] = half_dim(a2, N2);
    if (half) {
      nA = h[0].nL * N1 * N2;
      nB = h[0].nE * h[1].nL * N2;
      nC = h[0].nE * h[1].nE * h[2].nL;
      n = nA + nB + nC + h[0].nE * h[1].nE * h[2].nE;
    } else {
      nA = nB = nC = 0;
      n = N0 * N1 * N2;
    }
  }
  // coordinates of the i-th partner; returns 1 when its terms are doubled
  // (unsigned arithmetic: every index and extent here is non-negative, and
  // unsigned division by a run-time divisor is the shorter instruction
  // sequence)
  __device__ int get(int i_, int N1_, int N2_, int& b0, int& b1, int& b2) const {
    unsigned i = (unsigned)i_;
    const unsigned N2 = (unsigned)N2_, N12 = (unsigned)N1_ * N2;
    if (!half) {
      const unsigned j = i / N12, r = i - j * N12, k = r / N2;
      b0 = (int)j;
      b1 = (int)k;
      b2 = (int)(r - k * N2);
      return 0;
    }
    if (i < (unsigned)nA) {
      const unsigned j = i / N12, r = i - j * N12, k = r / N2;
      b0 = h[0].L((int)j);
      b1 = (int)k;
      b2 = (int)(r - k * N2);
      return 1;
    }
    i -= (unsigned)nA;
    if (i < (unsigned)nB) {
      const unsigned per = (unsigned)h[1].nL * N2, j = i / per, r = i - j * per, k = r / N2;
      b0 = h[0].E((int)j);
      b1 = h[1].L((int)k);
      b2 = (int)(r - k * N2);
      return 1;
    }
    i -= (unsigned)nB;
    if (i < (unsigned)nC) {
      const unsigned nL2 = (unsigned)h[2].nL, per = (unsigned)h[1].nE * nL2, j = i / per,
                     r = i - j * per, k = r / nL2;
      b0 = h[0].E((int)j);
      b1 = h[1].E((int)k);
      b2 = h[2].L((int)(r - k * nL2));
      return 1;
    }
    i -= (unsigned)nC;
    const unsigned nE2 = (unsigned)h[2].nE, per = (unsigned)h[1].nE * nE2, j = i / per,
                   r = i - j * per, k = r / nE2;
    b0 = h[0].E((int)j);
    b1 = h[1].E((int)k);
    b2 = h[2].E((int)(r - k * nE2));
    return 0;
  }
};

// Live q-points (a selected physical mode) in increasing order, the inverse
// map (-1 for the others) and their number.  One workgroup: thread t reads
// the flags of q = t + 1024 r for every round r first (coalesced, all loads
// in flight), then one block-wide scan per round orders the list.
// (A template only so that every translation unit that launches it may
// instantiate it from this header.)
template <int kUnused = 0>
__global__ __launch_bounds__(1024) void lw_live_q(int nq, int nb3, const uint8_t* __restrict__ phys,
                                                  const uint8_t* __restrict__ sel,
                                                  int32_t* __restrict__ list,
                                                  int32_t* __restrict__ idx_of_q,
                                                  int32_t* __restrict__ count) {
  __shared__ int wave_tot[2][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rounds = (nq + 1023) / 1024;  // <= 64 for N_q <= 65535
  unsigned long long live = 0;
  for (int r = 0; r < rounds; ++r) {
    const int q = tid + 1024 * r;
    int f = 0;
    if (q < nq)
      for (int s = 0; s < nb3; ++s) f |= phys[q * nb3 + s] & sel[q * nb3 + s];  // 0/1 bytes, no branch
    live |= (unsigned long long)f << r;
  }
  int carry = 0;
  for (int r = 0; r < rounds; ++r) {
    const int q = tid + 1024 * r;
    const int f = (int)(live >> r & 1ull);
    int incl = f;
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wave_tot[r & 1][wv] = incl;  // double-buffered: one barrier per round
    __syncthreads();
    int off = carry, tot = 0;
    for (int k = 0; k < 16; ++k) {
      off += (k < wv) ? wave_tot[r & 1][k] : 0;
      tot += wave_tot[r & 1][k];
    }
    if (q < nq) {
      idx_of_q[q] = f ? off + incl - 1 : -1;
      if (f) list[off + incl - 1] = q;
    }
    carry += tot;
  }
  if (tid == 0) *count = carry;
}

// Every q taken as live (all modes selected): identity list and map.  A q
// without a physical mode then gives only zero partial sums, which is what
// the finish kernels write for it anyway.
template <int kUnused = 0>
__global__ void lw_all_q(int nq, int32_t* __restrict__ list, int32_t* __restrict__ idx_of_q,
                         int32_t* __restrict__ count) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nq) {
    list[q] = q;
    idx_of_q[q] = q;
  }
  if (q == 0) *count = nq;
}

// Fused crystal kernel (lw_fused.hip): one workgroup per (q, chunk) work
// item, at most kFusedMaxChunks chunks per q, about `target` items in all.
constexpr int kFusedMaxChunks = 16;
constexpr int kWorkItems = 4096;  // (q, chunk) items a launch aims for
__host__ __device__ inline int fused_chunks(int n_live, int target) {
  if (n_live <= 0) return 1;
  const int c = (target + n_live - 1) / n_live;
  return c < 1 ? 1 : (c > kFusedMaxChunks ? kFusedMaxChunks : c);
}
bool fused_supported(const kaldo_crystal* c, int prec);
bool fused_record_supported(const kaldo_crystal* c, int prec);  // the cache's record pass

// What one launch of the fused kernel produces: Gamma (the linewidth sums),
// or, for the temperature cache, the number of cut-passing partner entries
// per (live q, chunk, branch) (count) and then the entries themselves
// (record).
enum FusedMode { kModeGamma = 0, kModeCount = 1, kModeRecord = 2 };
struct TcOut {
  long long* count;    // [n_live][kFusedMaxChunks][nb3], written by count, read by record
  long long* row_ptr;  // [n_modes + 1] row offsets per mode, written by count
  uint2* pairs;        // (m1, m2) of each entry, written by record
  double2* factors;    // (c, d) of each entry, written by record
  int32_t* flags;      // the handle's status word
};
template <typename T>
int launch_fused_cache(const kaldo_crystal* c, const LwParams& p, int mode, const double* omega,
                       const double* vel, const float4* modef, const double2* mrec,
                       const uint8_t* phys, const uint8_t* sel, const double* evec,
                       typename Cx<T>::type* eta, typename Cx<T>::type* phase_tab, int32_t* qlist,
                       int64_t n_subset, TcOut tc, hipStream_t st);
template <typename T>
int launch_fused(const kaldo_crystal* c, const LwParams& p, const double* omega, const double* vel,
                 const float4* modef, const double* occ, const double2* mrec, const uint8_t* phys,
                 const uint8_t* sel, const double* evec, typename Cx<T>::type* eta,
                 typename Cx<T>::type* phase_tab, int32_t* qlist, double* part, int64_t n_subset,
                 double scale, double* gamma, hipStream_t st);

// Dense MFMA crystal kernel (lw_mfma.hip).
bool mfma_supported(const kaldo_crystal* c);
int launch_mfma(const kaldo_crystal* c, const LwParams& p, bool split, const double* omega,
                const double* vel, const double* occ, const uint8_t* phys, const uint8_t* sel,
                const double* evec, float2* phase_tab, double scale, double* gamma,
                hipStream_t st);

}  // namespace kaldo
