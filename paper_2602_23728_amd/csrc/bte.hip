// Full scattering matrix of the linearised BTE and its two solutions
// (paper: "Boltzmann Transport Equation": Eq. BTE, Eq. gamma1, Eq. invBTE,
// Eq. kappa_general, Eq. sc_iter, Eq. inverse).
//
// Rows of Gamma~ = diag(Gamma0) + Gamma1, one per mode mu = (q, s).  For each
// ordered candidate (q s; q1 s'; q2 s''), q + q1 + q2 = G, passing the 2-sigma
// cut of the linewidths, with the coalescence and decay rates
//   d+ = 2 P |V|^2 (n1 - n2) g(x+) / (w w1 w2),
//   d- = 2 P |V|^2 1/2 (n1 + n2 + 1) g(x-) / (w w1 w2),   P = pi hbar U^3/(8 N_q),
// row mu receives Gamma0 += d+ + d- (= 2 Gamma of Eq. gamma), and
//   column (q1, s')       +d+ w1/w          (absorbed partner)
//   column tr(q1, s')     -d- w1/w          (emitted partner of the decay)
//   column tr(q2, s'')    -(d+ + d-) w2/w   (emitted partner of both)
// tr(q', s') is the time-reversal partner of a mode: the mode at -q' whose
// eigenvector overlaps eta(q', s')* most (the vertex holds eta(q2); the
// emitted phonon is the mode at -q2 with the conjugate eigenvector).  These
// rows make Eq. sc_iter the iterative scheme of the adaptive-smearing
// reference the paper cites.  Modes without RTA conductivity (nu < nu_min,
// Gamma0 <= 1e-8 max Gamma0) are decoupled: zero row and column, unit
// diagonal, zero right-hand side.
//
// Kernels:
//   bte_tr_map     time-reversal partner of every mode (largest overlap)
//   bte_zero       clears the n x n matrix
//   bte_rows<NB3>  one workgroup per q, three waves each over a third of
//                  the branches of q: A~_q (FP64, LDS, by atom block), then
//                  the partners q1 in rounds of 64 (one per lane): exact FP64
//                  cut, the passing candidates queued in the wave's LDS queue
//                  and their vertices computed by all its lanes, per-lane sums
//                  per column kind in LDS, written in three passes whose
//                  columns are a bijection of q1 (no two lanes of a pass touch
//                  one element), Gamma0 reduced in a fixed order and added to
//                  the diagonal
//   bte_gmax, bte_flags, bte_decouple   the RTA selection
//   bte_compact_index, bte_compact_cols, bte_gather3, bte_scatter3   the
//                  solve's restriction to the coupled modes (row map, coupled
//                  columns moved to the front of each coupled row)
//   lu_diag, lu_panels, lu_update, lu_gemm   blocked LU without pivoting of
//                  the coupled block (64 x 64 blocks, panels of eight; the
//                  panels and updates on the FP64 matrix cores)
//   lu_step<FORWARD>   the two triangular sweeps for the 3 RHS, one launch per block
//   bte_gemv, bte_sc_init, bte_sc_update   the iteration of Eq. sc_iter
//   bte_kappa      Eq. kappa_general, fixed-order reduction
// Every reduction and every sequence of additions into one matrix element
// runs in a fixed order: results are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "lw_common.h"

namespace kaldo {

constexpr int kLuB = 64;     // LU block edge
constexpr int kLuPanel = 8;  // blocks per panel of the blocked LU

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double d4;

// ------------------------------------------------------------------ tables

__global__ void bte_tr_map(int nq, int nb3, int N0, int N1, int N2,
                           const double* __restrict__ evec, int32_t* __restrict__ tr) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nq * nb3) return;
  const int q = m / nb3, s = m - q * nb3;
  const int a0 = q / (N1 * N2), a1 = (q / N2) % N1, a2 = q % N2;
  const int mq = (((N0 - a0) % N0) * N1 + (N1 - a1) % N1) * N2 + (N2 - a2) % N2;
  const double* x = evec + (size_t)q * nb3 * nb3 * 2;
  const double* y = evec + (size_t)mq * nb3 * nb3 * 2;
  int best = 0;
  double bo = -1.0;
  for (int t = 0; t < nb3; ++t) {
    double re = 0.0, im = 0.0;
    for (int i = 0; i < nb3; ++i) {
      const double xr = x[(i * nb3 + s) * 2], xi = x[(i * nb3 + s) * 2 + 1];
      const double yr = y[(i * nb3 + t) * 2], yi = y[(i * nb3 + t) * 2 + 1];
      re += yr * xr - yi * xi;  // eta_i(-q, t) eta_i(q, s), no conjugate
      im += yr * xi + yi * xr;
    }
    const double o = re * re + im * im;
    if (o > bo) {
      bo = o;
      best = t;
    }
  }
  tr[m] = mq * nb3 + best;
}

__global__ void bte_zero(size_t n, double* __restrict__ x) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    x[k] = 0.0;
}

// Per-process rates of one candidate without |V|^2 and the prefactor:
// dp = (n1 - n2) g(x+) / (w w1 w2), dm = 1/2 (n1 + n2 + 1) g(x-) / (w w1 w2),
// each 0 unless its own |x| < 2 sigma.
__device__ __forceinline__ void process_rates(const LwParams& p, double w, double w1, double w2,
                                              double n1, double n2, double sp, double sm,
                                              double& dp, double& dm) {
  const double xp = (w + w1) - w2, xm = (w - w1) - w2;
  const double den = w * (w1 * w2);
  dp = fabs(xp) < 2.0 * sp ? (n1 - n2) * smear(p.shape, xp, sp) / den : 0.0;
  dm = fabs(xm) < 2.0 * sm ? 0.5 * (n1 + n2 + 1.0) * smear(p.shape, xm, sm) / den : 0.0;
}

// ------------------------------------------------------------------ rows

constexpr int kRowWaves = 3;    // waves per row workgroup, each over a third of the branches s
constexpr int kRowQueue = 128;  // passing candidates a wave queues before projecting them

template <int NB3>
__global__ __launch_bounds__(64 * kRowWaves) void bte_rows(
    LwParams p, int n_rep, const int32_t* __restrict__ rep, const double* __restrict__ omega,
    const double* __restrict__ vel, const double* __restrict__ occ,
    const uint8_t* __restrict__ phys, const double* __restrict__ evec,
    const double2* __restrict__ phase_tab, int n_blk, const int32_t* __restrict__ e_blk,
    const int32_t* __restrict__ e_bg, const int32_t* __restrict__ blk_d,
    const int32_t* __restrict__ pair_ptr, const int32_t* __restrict__ t_ptr,
    const int32_t* __restrict__ t_i, const int32_t* __restrict__ t_l2,
    const double* __restrict__ t_coef, const int32_t* __restrict__ tr, double pref,
    double* __restrict__ mat, double* __restrict__ gamma0) {
  // [n_blk][9][NB3]: A~_q by atom block (jb, kb, d) and Cartesian pair
  // (beta, gamma), phases e^{+i q.R''} folded in
  extern __shared__ double2 at[];
  constexpr int NB = NB3 / 3;
  static_assert(NB3 % kRowWaves == 0, "the branches of q split evenly over the waves");
  constexpr int SPW = NB3 / kRowWaves;  // branches s per wave
  constexpr int BS = 64 * kRowWaves;
  __shared__ double acc[3][NB3][NB3][64];  // [kind][s][s' or s''][lane]
  __shared__ double2 phq[64];
  __shared__ double red[NB3][64];
  __shared__ int rq_code_w[kRowWaves][kRowQueue];  // lane | s1 << 6 | s2 << 12 | s << 18
  __shared__ double rq_dp_w[kRowWaves][kRowQueue], rq_dm_w[kRowWaves][kRowQueue],
      rq_v2_w[kRowWaves][kRowQueue];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int s_lo = wv * SPW;  // this wave's branches of q: [s_lo, s_lo + SPW)
  int* rq_code = rq_code_w[wv];
  double *rq_dp = rq_dp_w[wv], *rq_dm = rq_dm_w[wv], *rq_v2 = rq_v2_w[wv];
  const int q = blockIdx.x;
  const int nq = p.nq;
  const size_t n = (size_t)nq * NB3;
  const int N0 = p.N[0], N1 = p.N[1], N2 = p.N[2];
  const int a0 = q / (N1 * N2), a1 = (q / N2) % N1, a2 = q % N2;
  bool any = false;
  for (int s = 0; s < NB3; ++s) any = any || phys[q * NB3 + s];
  if (!any) {
    if (tid < NB3) gamma0[q * NB3 + tid] = 0.0;
    return;
  }
  for (int l = tid; l < n_rep; l += BS) {
    const int32_t* r = rep + 3 * l;
    const int m0 = ((a0 * r[0]) % N0 + N0) % N0, m1 = ((a1 * r[1]) % N1 + N1) % N1,
              m2 = ((a2 * r[2]) % N2 + N2) % N2;
    const double f = (double)m0 / N0 + (double)m1 / N1 + (double)m2 / N2;
    double sn, cs;
    sincospi(2.0 * f, &sn, &cs);
    phq[l] = make_double2(cs, sn);
  }
  for (int k = tid; k < n_blk * 9 * NB3; k += BS) at[k] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int k = tid; k < p.n_e * NB3; k += BS) {
    const int e = k / NB3, s = k % NB3;
    double re = 0.0, im = 0.0;
    for (int t = t_ptr[e]; t < t_ptr[e + 1]; ++t) {
      const size_t o = (((size_t)q * NB3 + t_i[t]) * NB3 + s) * 2;
      const double ex = evec[o], ey = evec[o + 1];
      const double2 f = phq[t_l2[t]];
      const double c = t_coef[t];
      re += c * (ex * f.x - ey * f.y);
      im += c * (ex * f.y + ey * f.x);
    }
    at[(e_blk[e] * 9 + e_bg[e]) * NB3 + s] = make_double2(re, im);
  }
  __syncthreads();
  double g0[NB3];
#pragma unroll
  for (int s = 0; s < NB3; ++s) g0[s] = 0.0;
  const int t0 = (N0 - a0) % N0, t1 = (N1 - a1) % N1, t2 = (N2 - a2) % N2;
  auto partner = [&](int q1) {
    const int b0 = q1 / (N1 * N2), b1 = (q1 / N2) % N1, b2 = q1 % N2;
    return (wrap_sub(t0, b0, N0) * N1 + wrap_sub(t1, b1, N1)) * N2 + wrap_sub(t2, b2, N2);
  };
  // |V|^2 of one (q1, s1, q2, s2, s) with the prefactor:
  // V = sum_blk e^{-i q1.R_d(blk)} sum_{beta gamma} A~[blk][beta gamma][s]
  //     eta_{3 jb + beta}(q1, s1) eta_{3 kb + gamma}(q2, s2),
  // the two eigenvector rows in registers, complex multiply-adds as fused
  // multiply-adds into the sums
  auto vertex2 = [&](int q1, int s1, int q2, int s2, int s) {
    double2 x[NB3], y[NB3];
#pragma unroll
    for (int i = 0; i < NB3; ++i) {
      const double* ex = evec + (((size_t)q1 * NB3 + i) * NB3 + s1) * 2;
      const double* ey = evec + (((size_t)q2 * NB3 + i) * NB3 + s2) * 2;
      x[i] = make_double2(ex[0], ex[1]);
      y[i] = make_double2(ey[0], ey[1]);
    }
    const double2* ph = phase_tab + (size_t)q1 * p.n_d;
    double vr = 0.0, vi = 0.0;
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
#pragma unroll
      for (int kb = 0; kb < NB; ++kb) {
        for (int blk = pair_ptr[jb * NB + kb]; blk < pair_ptr[jb * NB + kb + 1]; ++blk) {
          const double2* ab = at + (size_t)blk * 9 * NB3 + s;
          double ur = 0.0, ui = 0.0;
#pragma unroll
          for (int be = 0; be < 3; ++be) {
            double tr_ = 0.0, ti = 0.0;
#pragma unroll
            for (int ga = 0; ga < 3; ++ga) {
              const double2 a = ab[(be * 3 + ga) * NB3], v = y[3 * kb + ga];
              tr_ = fma(a.x, v.x, tr_);
              tr_ = fma(-a.y, v.y, tr_);
              ti = fma(a.x, v.y, ti);
              ti = fma(a.y, v.x, ti);
            }
            const double2 u = x[3 * jb + be];
            ur = fma(u.x, tr_, ur);
            ur = fma(-u.y, ti, ur);
            ui = fma(u.x, ti, ui);
            ui = fma(u.y, tr_, ui);
          }
          const double2 f = ph[blk_d[blk]];
          vr = fma(f.x, ur, vr);
          vr = fma(-f.y, ui, vr);
          vi = fma(f.x, ui, vi);
          vi = fma(f.y, ur, vi);
        }
      }
    }
    return pref * (vr * vr + vi * vi);
  };
  // A round takes 64 partners q1, one per lane of every wave; wave w takes
  // the branches s of q in [w SPW, (w + 1) SPW).  Each lane classifies its
  // (s1, s2, s) candidates in that order; the passing ones go to its wave's
  // queue in LDS (slots by ballot: candidate order, lanes ascending), whose
  // vertices all 64 lanes of the wave then compute; each lane then takes its
  // own entries back in queue order, so every sum sees the terms in the order
  // of the loops.  A wave's queue is its own: a wave-level fence and barrier
  // order its steps.
  const unsigned long long below = (1ull << lane) - 1ull;
  auto wave_sync = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  };
  for (int base = 0; base < nq; base += 64) {
    const int q1 = base + lane;
    const bool ok = q1 < nq;
    for (int k = 0; k < 3; ++k)
      for (int s = s_lo; s < s_lo + SPW; ++s)
        for (int u = 0; u < NB3; ++u) acc[k][s][u][lane] = 0.0;
    const int q2 = ok ? partner(q1) : 0;
    int qn = 0;  // entries in the queue (the same in every lane)
    auto flush = [&]() {
      wave_sync();
      for (int r = lane; r < qn; r += 64) {
        const int code = rq_code[r];
        const int o = code & 63, s1 = (code >> 6) & 63, s2 = (code >> 12) & 63, s = code >> 18;
        const int e1 = base + o;
        rq_v2[r] = vertex2(e1, s1, partner(e1), s2, s);
      }
      wave_sync();
      for (int r = 0; r < qn; ++r) {
        const int code = rq_code[r];
        if ((code & 63) != lane) continue;
        const int s1 = (code >> 6) & 63, s2 = (code >> 12) & 63, s = code >> 18;
        const double v2 = rq_v2[r];
        const double w = omega[q * NB3 + s], w1 = omega[q1 * NB3 + s1], w2 = omega[q2 * NB3 + s2];
        const double dp = rq_dp[r] * v2, dm = rq_dm[r] * v2;
        g0[s] += dp + dm;
        acc[0][s][s1][lane] += dp * (w1 / w);
        acc[1][s][s1][lane] += dm * (w1 / w);
        acc[2][s][s2][lane] += (dp + dm) * (w2 / w);
      }
      wave_sync();
      qn = 0;
    };
    for (int s1 = 0; s1 < NB3; ++s1) {
      const int m1 = q1 * NB3 + s1;
      const bool ok1 = ok && phys[m1];
      const double w1 = ok1 ? omega[m1] : 0.0, n1 = ok1 ? occ[m1] : 0.0;
      for (int s2 = 0; s2 < NB3; ++s2) {
        const int m2 = q2 * NB3 + s2;
        const bool ok2 = ok1 && phys[m2];
        double w2 = 0.0, n2 = 0.0, sp = 1.0, sm = 1.0;
        if (ok2) {
          w2 = omega[m2];
          n2 = occ[m2];
          widths(p, vel, m1, m2, sp, sm);
        }
        for (int s = s_lo; s < s_lo + SPW; ++s) {
          const int mu = q * NB3 + s;
          bool pass = false;
          double dp = 0.0, dm = 0.0;
          if (ok2 && phys[mu]) {
            const double w = omega[mu];
            // the cut first (most candidates fail it), then the rates
            if (fabs((w + w1) - w2) < 2.0 * sp || fabs((w - w1) - w2) < 2.0 * sm) {
              process_rates(p, w, w1, w2, n1, n2, sp, sm, dp, dm);
              pass = !(dp == 0.0 && dm == 0.0);
            }
          }
          const unsigned long long mask = __ballot(pass);
          if (mask == 0ull) continue;
          if (qn + __popcll(mask) > kRowQueue) flush();
          if (pass) {
            const int r = qn + __popcll(mask & below);
            rq_code[r] = lane | (s1 << 6) | (s2 << 12) | (s << 18);
            rq_dp[r] = dp;
            rq_dm[r] = dm;
          }
          qn += __popcll(mask);
        }
      }
    }
    flush();
    __syncthreads();
    // three passes; within each the columns of different lanes differ
    if (ok) {
      for (int s = s_lo; s < s_lo + SPW; ++s) {
        double* row = mat + (size_t)(q * NB3 + s) * n;
        for (int u = 0; u < NB3; ++u) {
          const double x = acc[0][s][u][lane];
          if (x != 0.0) row[q1 * NB3 + u] += x;
        }
      }
    }
    __syncthreads();
    if (ok) {
      for (int s = s_lo; s < s_lo + SPW; ++s) {
        double* row = mat + (size_t)(q * NB3 + s) * n;
        for (int u = 0; u < NB3; ++u) {
          const double x = acc[1][s][u][lane];
          if (x != 0.0) row[tr[q1 * NB3 + u]] -= x;
        }
      }
    }
    __syncthreads();
    if (ok) {
      for (int s = s_lo; s < s_lo + SPW; ++s) {
        double* row = mat + (size_t)(q * NB3 + s) * n;
        for (int u = 0; u < NB3; ++u) {
          const double x = acc[2][s][u][lane];
          if (x != 0.0) row[tr[q2 * NB3 + u]] -= x;
        }
      }
    }
    __syncthreads();
  }
  // Gamma0: fixed-order tree over the lanes, then onto the diagonal
  for (int s = s_lo; s < s_lo + SPW; ++s) red[s][lane] = g0[s];
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (lane < w)
      for (int s = s_lo; s < s_lo + SPW; ++s) red[s][lane] += red[s][lane + w];
    __syncthreads();
  }
  if (lane < SPW) {
    const int s = s_lo + lane, mu = q * NB3 + s;
    const double g = phys[mu] ? red[s][0] : 0.0;
    gamma0[mu] = g;
    mat[(size_t)mu * n + mu] += g;
  }
}

// Largest Gamma0 (order-independent), one workgroup.
__global__ __launch_bounds__(1024) void bte_gmax(long n, const double* __restrict__ g0,
                                                 double* __restrict__ out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (long k = threadIdx.x; k < n; k += 1024) m = fmax(m, g0[k]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__device__ __forceinline__ bool bte_active(double w, double g, double gmax, double nu_min) {
  return (w / kTwoPi >= nu_min) && (g > kGammaFloorRel * gmax) && (g > 0.0);
}

// Which modes keep their RTA conductivity (1) or are decoupled (0).
__global__ void bte_flags(long n, const double* __restrict__ omega, const double* __restrict__ g0,
                          const double* __restrict__ gmax, double nu_min,
                          uint8_t* __restrict__ act) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) act[i] = bte_active(omega[i], g0[i], *gmax, nu_min) ? 1 : 0;
}

// Decoupled modes: zero row and column, unit diagonal.  One workgroup per
// row j, its threads along the row: a decoupled row is written whole, the
// row of a kept mode only at the decoupled columns (coalesced either way).
__global__ __launch_bounds__(256) void bte_decouple(long n, const uint8_t* __restrict__ act,
                                                    double* __restrict__ mat) {
  const long j = blockIdx.x;
  if (j >= n) return;
  double* row = mat + j * n;
  if (!act[j]) {
    for (long i = threadIdx.x; i < n; i += 256) row[i] = (i == j) ? 1.0 : 0.0;
  } else {
    for (long i = threadIdx.x; i < n; i += 256)
      if (!act[i]) row[i] = 0.0;
  }
}

// Right-hand side: v on active modes, 0 elsewhere; rhs[i][3].
// The coupled modes in order: rows[a] = the a-th mode with act = 1, *count =
// their number.  One workgroup; each thread counts a contiguous run of
// modes, a block-wide scan places the runs.
__global__ __launch_bounds__(1024) void bte_compact_index(long n, const uint8_t* __restrict__ act,
                                                          int32_t* __restrict__ rows,
                                                          int32_t* __restrict__ count) {
  __shared__ int sums[1024];
  const int tid = threadIdx.x;
  const long per = (n + 1023) / 1024;
  const long lo = tid * per < n ? tid * per : n, hi = lo + per < n ? lo + per : n;
  int c = 0;
  for (long i = lo; i < hi; ++i) c += act[i];
  sums[tid] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = tid >= off ? sums[tid - off] : 0;
    __syncthreads();
    sums[tid] += v;
    __syncthreads();
  }
  int r = sums[tid] - c;
  for (long i = lo; i < hi; ++i)
    if (act[i]) rows[r++] = (int32_t)i;
  if (tid == 1023) *count = sums[1023];
}

// Moves the coupled columns of a coupled row to its front: row rows[a]
// becomes (A[rows[a]][rows[0]], ..., A[rows[a]][rows[na - 1]], ...).  One
// workgroup per row, in slices of 256 columns: a slice's values are all read
// before any is written, and its targets lie before the sources of every
// later slice (rows[b] >= b).
__global__ __launch_bounds__(256) void bte_compact_cols(long na, long ld,
                                                        const int32_t* __restrict__ rows,
                                                        double* __restrict__ mat) {
  const long a = blockIdx.x;
  if (a >= na) return;
  double* row = mat + (long)rows[a] * ld;
  for (long b0 = 0; b0 < na; b0 += 256) {
    const long b = b0 + threadIdx.x;
    const double v = b < na ? row[rows[b]] : 0.0;
    __syncthreads();
    if (b < na) row[b] = v;
    __syncthreads();
  }
}

// dst[a] = src[rows[a]] (three components), and back: dst[rows[a]] = src[a]
// over a zeroed dst.
__global__ void bte_gather3(long na, const int32_t* __restrict__ rows,
                            const double* __restrict__ src, double* __restrict__ dst) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 3 * na) dst[k] = src[3 * (long)rows[k / 3] + k % 3];
}
__global__ void bte_scatter3(long na, const int32_t* __restrict__ rows,
                             const double* __restrict__ src, double* __restrict__ dst) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 3 * na) dst[3 * (long)rows[k / 3] + k % 3] = src[k];
}

__global__ void bte_rhs(long n, const double* __restrict__ omega, const double* __restrict__ vel,
                        const double* __restrict__ g0, const double* __restrict__ gmax,
                        double nu_min, double* __restrict__ rhs) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool a = bte_active(omega[i], g0[i], *gmax, nu_min);
  for (int c = 0; c < 3; ++c) rhs[3 * i + c] = a ? vel[3 * i + c] : 0.0;
}

// kappa_ab = scale sum_i c_i v_ia lambda_ib over active modes; one workgroup.
__global__ __launch_bounds__(1024) void bte_kappa(long n, const double* __restrict__ omega,
                                                  const double* __restrict__ vel,
                                                  const double* __restrict__ lam,
                                                  const double* __restrict__ g0,
                                                  const double* __restrict__ gmax,
                                                  double inv_kt_hbar, double nu_min,
                                                  double scale, double* __restrict__ kappa) {
  __shared__ double red[1024][9];
  const int t = threadIdx.x;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const double gm = *gmax;
  for (long i = t; i < n; i += 1024) {
    const double w = omega[i];
    if (!bte_active(w, g0[i], gm, nu_min)) continue;
    const double x = w * inv_kt_hbar;
    const double em = expm1(x);
    const double c = x * x * (em + 1.0) / (em * em);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) acc[3 * a + b] += c * vel[3 * i + a] * lam[3 * i + b];
  }
  for (int k = 0; k < 9; ++k) red[t][k] = acc[k];
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w)
      for (int k = 0; k < 9; ++k) red[t][k] += red[t + w][k];
    __syncthreads();
  }
  if (t < 9) kappa[t] = scale * red[0][t];
}

// ------------------------------------------------------------------ LU

// Factor the diagonal block k (no pivoting) in LDS; write L\U back, and the
// inverses of the unit lower L and of the upper U to linv/uinv [64][64].
// Padding rows past n act as identity rows.
// The coupled block of the matrix as the LU sees it: element (i, j) of the
// n x n coupled system sits at row rows[i] of the stored matrix (leading
// dimension ld), column j (the coupled columns of each stored row are moved
// to its front by bte_compact_cols).
struct MatRows {
  double* mat;
  const int32_t* rows;
  long ld;
  __device__ double* row(long i) const { return mat + (long)rows[i] * ld; }
};

__global__ __launch_bounds__(256) void lu_diag(long n, int k, MatRows A,
                                               double* __restrict__ linv,
                                               double* __restrict__ uinv,
                                               int32_t* __restrict__ flags) {
  // Thread (ty, tx) = (tid / 16, tid % 16) keeps in registers the 16
  // elements of rows ty + 16 a and columns tx + 16 b (a, b < 4) of the block
  // D, of X_L = L^-1 and of X_U = U^-1: the strided split keeps every thread
  // busy as the active corner shrinks.  Step j publishes through LDS the
  // rows and columns it needs (two buffers by step parity, so one barrier
  // per step); then, with r = 1 / D[j][j] and l_i = D[i][j] r:
  //   factorisation        D[i][c] -= l_i D[j][c]          (i, c > j), D[i][j] = l_i
  //   unit lower inverse   X_L[i][:] -= l_i X_L[j][:]      (i > j; row j of X_L is final)
  //   upper inverse        X_U[:][j] *= r, then X_U[:][c] -= X_U[:][j] U[j][c]   (c > j)
  // Row j of D is row j of U from step j on, and column j of X_U has then
  // taken every earlier step, so all three run in the same 64 steps.
  constexpr int B = kLuB;
  static_assert(B == 64, "16 x 16 threads, 4 x 4 elements each");
  __shared__ double pub_row[2][B];    // row j of D
  __shared__ double pub_col[2][B];    // column j of D
  __shared__ double pub_xrow[2][B];   // row j of X_L
  __shared__ double pub_xucol[2][B];  // column j of X_U
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  const long r0 = (long)k * B;
  double d[4][4], xl[4][4], xu[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ty + 16 * a, c = tx + 16 * b;
      const long gi = r0 + i, gc = r0 + c;
      d[a][b] = (gi < n && gc < n) ? A.row(gi)[gc] : (i == c ? 1.0 : 0.0);
      xl[a][b] = xu[a][b] = (i == c) ? 1.0 : 0.0;
    }
#pragma unroll
  for (int ja = 0; ja < 4; ++ja) {
    for (int jy = 0; jy < 16; ++jy) {
      const int j = 16 * ja + jy, pb = j & 1;
      if (ty == jy) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          pub_row[pb][tx + 16 * b] = d[ja][b];
          pub_xrow[pb][tx + 16 * b] = xl[ja][b];
        }
      }
      if (tx == jy) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          pub_col[pb][ty + 16 * a] = d[a][ja];
          pub_xucol[pb][ty + 16 * a] = xu[a][ja];
        }
      }
      __syncthreads();
      const double piv = pub_row[pb][j];
      if (tid == 0 && !(fabs(piv) > 1e-300)) raise_flag(flags, kFlagSingular);
      const double r = 1.0 / piv;
      double uc[4], xc[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        uc[b] = pub_row[pb][tx + 16 * b];
        xc[b] = pub_xrow[pb][tx + 16 * b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int i = ty + 16 * a;
        const double xj = pub_xucol[pb][i] * r;
        const double li = pub_col[pb][i] * r;
        const bool below = i > j;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int c = tx + 16 * b;
          if (c > j) {
            if (below) d[a][b] = fma(-li, uc[b], d[a][b]);
            xu[a][b] = fma(-xj, uc[b], xu[a][b]);
          }
          if (b == ja && c == j) {
            if (below) d[a][b] = li;
            xu[a][b] = xj;
          }
          if (below) xl[a][b] = fma(-li, xc[b], xl[a][b]);
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ty + 16 * a, c = tx + 16 * b;
      const long gi = r0 + i, gc = r0 + c;
      if (gi < n && gc < n) A.row(gi)[gc] = d[a][b];
      linv[i * B + c] = xl[a][b];
      uinv[i * B + c] = xu[a][b];
    }
}

// 64 x 64 x 64 product P Q from two LDS blocks, four waves of 32 x 32 on
// v_mfma_f64_16x16x4f64; wave wv holds rows wm = 32 (wv / 2) and columns
// wn = 32 (wv % 2) of the result in acc[a][b] (16 x 16 tiles).
struct BlockProduct {
  int wm, wn, lr, lg;
  d4 acc[2][2];
  __device__ void run(const double (*P)[kLuB + 1], const double (*Q)[kLuB + 1], int tid) {
    const int lane = tid & 63, wv = tid >> 6;
    wm = (wv >> 1) * 32;
    wn = (wv & 1) * 32;
    lr = lane & 15;
    lg = lane >> 4;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < kLuB; kk += 4) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const double av = P[wm + 16 * a + lr][kk + lg];  // A[row = lane % 16][k = lane / 16]
          const double bv = Q[kk + lg][wn + 16 * b + lr];  // B[k = lane / 16][col = lane % 16]
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[a][b], 0, 0, 0);
        }
    }
  }
  // FP64 16 x 16 accumulator: item r of lane l is row 4 r + l / 16, column l % 16
  __device__ int row(int a, int r) const { return wm + 16 * a + 4 * r + lg; }
  __device__ int col(int b) const { return wn + 16 * b + lr; }
};

// Panels of step k: row blocks A_kj <- Linv A_kj (j > k, first nb - k - 1
// workgroups), column blocks A_ik <- A_ik Uinv (i > k, the rest).
__global__ __launch_bounds__(256) void lu_panels(long n, int nb, int k, MatRows A,
                                                 const double* __restrict__ linv,
                                                 const double* __restrict__ uinv) {
  constexpr int B = kLuB;
  __shared__ double M[B][B + 1];
  __shared__ double T[B][B + 1];
  const int tid = threadIdx.x;
  const int m = nb - k - 1;
  const bool row = (int)blockIdx.x < m;
  const int other = k + 1 + (row ? blockIdx.x : blockIdx.x - m);
  const long bi = row ? k : other, bj = row ? other : k;
  for (int idx = tid; idx < B * B; idx += 256) {
    const int i = idx / B, j = idx % B;
    const long gi = bi * B + i, gj = bj * B + j;
    M[i][j] = (gi < n && gj < n) ? A.row(gi)[gj] : 0.0;
    T[i][j] = row ? linv[idx] : uinv[idx];
  }
  __syncthreads();
  BlockProduct bp;
  if (row)
    bp.run(T, M, tid);
  else
    bp.run(M, T, tid);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long gi = bi * B + bp.row(a, r), gj = bj * B + bp.col(b);
        if (gi < n && gj < n) A.row(gi)[gj] = bp.acc[a][b][r];
      }
}

// Update of step k on two rectangles of blocks: A_ij -= A_ik A_kj for i in
// [i0, i0 + ni), j in [j0, j0 + nj) (the first n1 workgroups), then for i in
// [i0b, ...), j in [j0b, j0b + njb); one 64 x 64 block per workgroup.  The
// rectangles are disjoint and read only row and column k.
__global__ __launch_bounds__(256) void lu_update(long n, int k, int i0, int j0, int nj, int n1,
                                                 int i0b, int j0b, int njb, MatRows A) {
  constexpr int B = kLuB;
  __shared__ double L[B][B + 1];
  __shared__ double U[B][B + 1];
  const int tid = threadIdx.x;
  const int wb = (int)blockIdx.x;
  const long bi = wb < n1 ? i0 + wb / nj : i0b + (wb - n1) / njb,
             bj = wb < n1 ? j0 + wb % nj : j0b + (wb - n1) % njb;
  for (int idx = tid; idx < B * B; idx += 256) {
    const int i = idx / B, j = idx % B;
    const long li = bi * B + i, lj = (long)k * B + j;
    L[i][j] = (li < n && lj < n) ? A.row(li)[lj] : 0.0;
    const long ui = (long)k * B + i, uj = bj * B + j;
    U[i][j] = (ui < n && uj < n) ? A.row(ui)[uj] : 0.0;
  }
  __syncthreads();
  BlockProduct bp;
  bp.run(L, U, tid);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long gi = bi * B + bp.row(a, r), gj = bj * B + bp.col(b);
        if (gi < n && gj < n) A.row(gi)[gj] -= bp.acc[a][b][r];
      }
}

// Deferred update of a panel: A_ij -= sum_k A_ik A_kj over the panel's
// columns k in [kc, kc + kw) for the trailing elements i, j >= r0 (blocked
// right-looking LU: the panel's own steps update only the panel's columns
// and rows, this one product the rest).  128 x 128 tile per workgroup, four
// waves of 64 x 64 as 4 x 4 v_mfma_f64_16x16x4f64 accumulators; K in slices
// of 16 staged k-major in LDS (two buffers, the next slice fetched into
// registers while the current one is multiplied).  Elements past n read as
// zero and are not written.
constexpr int kLgT = 128;  // tile edge
constexpr int kLgK = 16;   // K slice
constexpr int kLgLd = kLgT + 2;  // LDS row stride (doubles)

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void lu_gemm(long n, long r0, long kc, int kw, int ntl,
                                               MatRows A) {
  __shared__ double As[2][kLgK][kLgLd];  // [k][row]
  __shared__ double Bs[2][kLgK][kLgLd];  // [k][col]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const long row0 = r0 + (long)(blockIdx.x / ntl) * kLgT, col0 = r0 + (long)(blockIdx.x % ntl) * kLgT;
  if (row0 >= n || col0 >= n) return;
  // staging: A rows row0 + (tid >> 1), k = 8 (tid & 1) .. + 8; B row k =
  // tid >> 4, columns col0 + 8 (tid & 15) .. + 8
  const int ar = tid >> 1, ak = 8 * (tid & 1);
  const int bk = tid >> 4, bc = 8 * (tid & 15);
  const long ga = row0 + ar, gbc = col0 + bc;
  const double* arow = A.row(ga < n ? ga : 0);  // row ga (a valid row when ga >= n)
  double pa[8], pb[8];
  // slice k0: eight consecutive elements per operand and thread, from one
  // base address (constant offsets)
  auto fetch = [&](long k0) {
    const long ka = k0 + ak;
    const double* a = arow + ka;
#pragma unroll
    for (int t = 0; t < 8; ++t) pa[t] = (ga < n && ka + t < n) ? a[t] : 0.0;
    const long kb = k0 + bk;
    const double* b = A.row(kb < n ? kb : 0) + gbc;
#pragma unroll
    for (int t = 0; t < 8; ++t) pb[t] = (kb < n && gbc + t < n) ? b[t] : 0.0;
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int t = 0; t < 8; ++t) As[buf][ak + t][ar] = pa[t];
#pragma unroll
    for (int t = 0; t < 8; ++t) Bs[buf][bk][bc + t] = pb[t];
  };
  const int wm = (wv >> 1) * 64, wn = (wv & 1) * 64;
  const int lr = lane & 15, lg = lane >> 4;
  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  fetch(kc);
  stage(0);
  __syncthreads();
  int cur = 0;
  for (long k0 = kc; k0 < kc + kw; k0 += kLgK) {
    const bool more = k0 + kLgK < kc + kw;
    if (more) fetch(k0 + kLgK);
#pragma unroll
    for (int kk = 0; kk < kLgK; kk += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        av[t] = As[cur][kk + lg][wm + 16 * t + lr];  // A[row = lane % 16][k = lane / 16]
        bv[t] = Bs[cur][kk + lg][wn + 16 * t + lr];  // B[k = lane / 16][col = lane % 16]
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (more) stage(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // item r of lane l is row 4 r + l / 16, column l % 16
        const long gi = row0 + wm + 16 * a + 4 * r + lg, gj = col0 + wn + 16 * b + lr;
        if (gi < n && gj < n) A.row(gi)[gj] -= acc[a][b][r];
      }
}

// Triangular sweeps with 3 right-hand sides, right-looking: the residual r
// starts as the right-hand side; step k solves block k, x_k = Tinv_k r_k,
// and removes its contribution from the blocks still to solve, r_i -= A_ik
// x_k (i > k forward with the L blocks, i < k backward with the U blocks),
// in one launch: every workgroup forms x_k in LDS, workgroup 0 stores it and
// each other one updates one block.  Every r_i is updated in the order of k:
// the sums are fixed-order.
template <bool FORWARD>
__global__ __launch_bounds__(256) void lu_step(long n, int k, const double* __restrict__ tinv,
                                               MatRows A, double* __restrict__ x,
                                               double* __restrict__ r) {
  constexpr int B = kLuB;
  __shared__ double rk[B][3];
  __shared__ double xk[B][3];
  __shared__ double part[4][B][3];
  const int tid = threadIdx.x, row = tid >> 2, sub = tid & 3;
  if (tid < B * 3) {
    const int i = tid / 3, c = tid % 3;
    const long g = (long)k * B + i;
    rk[i][c] = g < n ? r[3 * g + c] : 0.0;
  }
  __syncthreads();
  if (tid < B * 3) {
    const int i = tid / 3, c = tid % 3;
    double s = 0.0;
    for (int t = 0; t < B; ++t) s += tinv[i * B + t] * rk[t][c];
    xk[i][c] = s;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid < B * 3) {
      const int i = tid / 3, c = tid % 3;
      const long g = (long)k * B + i;
      if (g < n) x[3 * g + c] = xk[i][c];
    }
    return;
  }
  const long bi = FORWARD ? k + (long)blockIdx.x : (long)blockIdx.x - 1;
  const long gi = bi * B + row;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (gi < n)
    for (int t = sub; t < B; t += 4) {
      const long gc = (long)k * B + t;
      if (gc >= n) break;
      const double a = A.row(gi)[gc];
      s0 += a * xk[t][0];
      s1 += a * xk[t][1];
      s2 += a * xk[t][2];
    }
  part[sub][row][0] = s0;
  part[sub][row][1] = s1;
  part[sub][row][2] = s2;
  __syncthreads();
  if (tid < B * 3) {
    const int i = tid / 3, c = tid % 3;
    const long g = bi * B + i;
    if (g < n) r[3 * g + c] -= ((part[0][i][c] + part[1][i][c]) + part[2][i][c]) + part[3][i][c];
  }
}

__global__ void bte_copy3(long n, const double* __restrict__ src, double* __restrict__ dst) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * n) dst[i] = src[i];
}

// ------------------------------------------------------------------ iteration

// y = A x for 3 right-hand sides, one workgroup per row, fixed-order sums.
__global__ __launch_bounds__(256) void bte_gemv(long n, const double* __restrict__ mat,
                                                const double* __restrict__ x,
                                                double* __restrict__ y) {
  __shared__ double red[256][3];
  const long i = blockIdx.x;
  const int t = threadIdx.x;
  const double* a = mat + i * n;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (long c = t; c < n; c += 256) {
    const double v = a[c];
    s0 += v * x[3 * c];
    s1 += v * x[3 * c + 1];
    s2 += v * x[3 * c + 2];
  }
  red[t][0] = s0;
  red[t][1] = s1;
  red[t][2] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int c = 0; c < 3; ++c) red[t][c] += red[t + w][c];
    __syncthreads();
  }
  if (t < 3) y[3 * i + t] = red[0][t];
}

// lambda0 = v / Gamma0 on active modes (Eq. sc_iter's start, the RTA).
__global__ void bte_sc_init(long n, const double* __restrict__ rhs, const double* __restrict__ g0,
                            double* __restrict__ lam) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool a = rhs[3 * i] != 0.0 || rhs[3 * i + 1] != 0.0 || rhs[3 * i + 2] != 0.0;
  for (int c = 0; c < 3; ++c) lam[3 * i + c] = a ? rhs[3 * i + c] / g0[i] : 0.0;
}

// lambda <- (v - Gamma1 lambda) / Gamma0 = lambda + (v - Gamma~ lambda) / Gamma0
// (y = Gamma~ lambda); decoupled modes keep lambda = 0.
__global__ void bte_sc_update(long n, const double* __restrict__ rhs,
                              const double* __restrict__ g0, const double* __restrict__ omega,
                              const double* __restrict__ gmax, double nu_min,
                              const double* __restrict__ y, double* __restrict__ lam) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!bte_active(omega[i], g0[i], *gmax, nu_min)) return;
  for (int c = 0; c < 3; ++c) lam[3 * i + c] += (rhs[3 * i + c] - y[3 * i + c]) / g0[i];
}

// ------------------------------------------------------------------ host

struct BteWs {
  size_t off_occ, off_phys, off_act, off_rows, off_count, off_tr, off_phase, off_gmax, off_rhs,
      off_lam, off_y, off_y2,
      off_linv, off_uinv, off_kappa, total;
};

static BteWs bte_ws(const kaldo_crystal* c, long nq) {
  const long n = nq * c->nb3;
  const long nb = (n + kLuB - 1) / kLuB;
  BteWs w;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  w.off_occ = take(8 * n);
  w.off_phys = take(n);
  w.off_act = take(n);
  w.off_rows = take(4 * n);
  w.off_count = take(4);
  w.off_tr = take(4 * n);
  w.off_phase = take(16 * nq * (size_t)std::max(1, c->bloch.n_d));
  w.off_gmax = take(8);
  w.off_rhs = take(24 * n);
  w.off_lam = take(24 * n);
  w.off_y = take(24 * n);
  w.off_y2 = take(24 * n);
  w.off_linv = take(8 * kLuB * kLuB * nb);
  w.off_uinv = take(8 * kLuB * kLuB * nb);
  w.off_kappa = take(8 * 9);
  w.total = o;
  return w;
}

static bool bte_supported(const kaldo_crystal* c) {
  if (c->nb3 != 3 && c->nb3 != 6) return false;
  return (size_t)c->bloch.n_blk * 9 * c->nb3 * 16 <= 64 * 1024 && c->n_rep <= 64;
}

__global__ void bte_prepare(int n_modes, const double* __restrict__ omega, double inv_kt_hbar,
                            double nu_min, double* __restrict__ occ, uint8_t* __restrict__ phys,
                            int32_t* __restrict__ flags) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_modes) return;
  const double w = omega[m];
  const bool p = (w / kTwoPi) >= nu_min;
  phys[m] = p;
  occ[m] = p ? 1.0 / expm1(w * inv_kt_hbar) : 0.0;
  if (!(w - w == 0.0)) raise_flag(flags, kFlagNonFinite);
  if (w < 0.0 && (-w / kTwoPi) >= nu_min) raise_flag(flags, kFlagImaginary);
}

static int check_common(const kaldo_crystal* c, const int32_t* mesh, double T, long* nq_out) {
  KALDO_REQUIRE(c && mesh, "bte: NULL argument");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "bte: mesh must be >= 1");
  KALDO_REQUIRE(std::isfinite(T) && T > 0, "bte: temperature <= 0");
  const long nq = (long)mesh[0] * mesh[1] * mesh[2];
  KALDO_REQUIRE(nq <= 65535L, "bte: mesh too large (N_q > 65535)");
  *nq_out = nq;
  return KALDO_OK;
}

}  // namespace kaldo

using namespace kaldo;

extern "C" size_t kaldo_bte_workspace(const kaldo_crystal* c, const int32_t* mesh) {
  if (!c || !mesh || mesh[0] < 1 || mesh[1] < 1 || mesh[2] < 1) return 0;
  return bte_ws(c, (long)mesh[0] * mesh[1] * mesh[2]).total;
}

extern "C" int kaldo_scattering_matrix(const kaldo_crystal* c, const int32_t* mesh,
                                       const double* omega, const double* evec, const double* vel,
                                       double temperature, const kaldo_broadening* b,
                                       void* workspace, size_t workspace_bytes, double* matrix,
                                       double* gamma0, void* stream) {
  long nq = 0;
  int rc = check_common(c, mesh, temperature, &nq);
  if (rc) return rc;
  KALDO_REQUIRE(omega && evec && vel && b && matrix && gamma0, "kaldo_scattering_matrix: NULL argument");
  rc = check_broadening(b, true);
  if (rc) return rc;
  if (!bte_supported(c)) {
    set_error("kaldo_scattering_matrix: implemented for cells of 1 or 2 atoms whose folded FC3 fits 64 KB of LDS");
    return KALDO_EUNSUPPORTED;
  }
  const BteWs w = bte_ws(c, nq);
  KALDO_REQUIRE(workspace && workspace_bytes >= w.total, "kaldo_scattering_matrix: workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto* ws = static_cast<unsigned char*>(workspace);
  const int nb3 = c->nb3;
  const long n = nq * nb3;
  double* occ = reinterpret_cast<double*>(ws + w.off_occ);
  uint8_t* phys = ws + w.off_phys;
  uint8_t* act = ws + w.off_act;
  int32_t* tr = reinterpret_cast<int32_t*>(ws + w.off_tr);
  double2* phase = reinterpret_cast<double2*>(ws + w.off_phase);
  double* gmax = reinterpret_cast<double*>(ws + w.off_gmax);
  LwParams p = make_params(c, mesh, temperature, b);
  KALDO_LAUNCH("bte_prepare", bte_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
               (int)n, omega, kHbar / (kKb * temperature), b->nu_min_thz, occ, phys, c->d_flags);
  KALDO_LAUNCH("bte_tr_map", bte_tr_map, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
               (int)nq, nb3, mesh[0], mesh[1], mesh[2], evec, tr);
  const long nph = nq * std::max(1, p.n_d);
  KALDO_LAUNCH("lw_phase_table", lw_phase_table<double>, dim3((unsigned)((nph + 255) / 256)),
               dim3(256), 0, st, (int)nq, p.n_d, mesh[0], mesh[1], mesh[2], c->bloch.dvec, phase);
  const size_t n2 = (size_t)n * n;
  KALDO_LAUNCH("bte_zero", bte_zero, dim3((unsigned)std::min<size_t>((n2 + 255) / 256, 1u << 20)),
               dim3(256), 0, st, n2, matrix);
  const size_t lds = (size_t)c->bloch.n_blk * 9 * nb3 * sizeof(double2);
  const double pref = 2.0 * kPrefactor / (double)nq;
  const Fc3Bloch& bl = c->bloch;
  if (nb3 == 6)
    KALDO_LAUNCH("bte_rows", bte_rows<6>, dim3((unsigned)nq), dim3(64 * kRowWaves), lds, st, p, c->n_rep,
                 c->d_rep, omega, vel, occ, phys, evec, phase, bl.n_blk, bl.e_blk, bl.e_bg,
                 bl.blk_d, bl.pair_ptr, bl.t_ptr, bl.t_i, bl.t_l2, bl.t_coef, tr, pref, matrix,
                 gamma0);
  else
    KALDO_LAUNCH("bte_rows", bte_rows<3>, dim3((unsigned)nq), dim3(64 * kRowWaves), lds, st, p, c->n_rep,
                 c->d_rep, omega, vel, occ, phys, evec, phase, bl.n_blk, bl.e_blk, bl.e_bg,
                 bl.blk_d, bl.pair_ptr, bl.t_ptr, bl.t_i, bl.t_l2, bl.t_coef, tr, pref, matrix,
                 gamma0);
  KALDO_LAUNCH("bte_gmax", bte_gmax, dim3(1), dim3(1024), 0, st, n, gamma0, gmax);
  KALDO_LAUNCH("bte_flags", bte_flags, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
               omega, gamma0, gmax, b->nu_min_thz, act);
  KALDO_LAUNCH("bte_decouple", bte_decouple, dim3((unsigned)n), dim3(256), 0, st, n, act, matrix);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

static int bte_solve_common(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                            const double* vel, const double* gamma0, double T, double nu_min,
                            void* workspace, size_t workspace_bytes, const BteWs& w, long nq,
                            hipStream_t st) {
  KALDO_REQUIRE(omega && vel && gamma0, "bte: NULL argument");
  KALDO_REQUIRE(std::isfinite(nu_min) && nu_min >= 0, "bte: nu_min_thz < 0");
  KALDO_REQUIRE(workspace && workspace_bytes >= w.total, "bte: workspace too small");
  auto* ws = static_cast<unsigned char*>(workspace);
  const long n = nq * c->nb3;
  double* gmax = reinterpret_cast<double*>(ws + w.off_gmax);
  double* rhs = reinterpret_cast<double*>(ws + w.off_rhs);
  (void)mesh;
  (void)T;
  KALDO_LAUNCH("bte_gmax", bte_gmax, dim3(1), dim3(1024), 0, st, n, gamma0, gmax);
  KALDO_LAUNCH("bte_rhs", bte_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, omega,
               vel, gamma0, gmax, nu_min, rhs);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_bte_solve(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                               const double* vel, const double* gamma0, double temperature,
                               double nu_min_thz, double* matrix, void* workspace,
                               size_t workspace_bytes, double* lambda, double* kappa,
                               void* stream) {
  long nq = 0;
  int rc = check_common(c, mesh, temperature, &nq);
  if (rc) return rc;
  KALDO_REQUIRE(matrix && lambda && kappa, "kaldo_bte_solve: NULL argument");
  const BteWs w = bte_ws(c, nq);
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = bte_solve_common(c, mesh, omega, vel, gamma0, temperature, nu_min_thz, workspace,
                        workspace_bytes, w, nq, st);
  if (rc) return rc;
  auto* ws = static_cast<unsigned char*>(workspace);
  const long n_all = nq * c->nb3;
  double* linv = reinterpret_cast<double*>(ws + w.off_linv);
  double* uinv = reinterpret_cast<double*>(ws + w.off_uinv);
  double* rhs = reinterpret_cast<double*>(ws + w.off_rhs);
  double* lam_c = reinterpret_cast<double*>(ws + w.off_lam);
  double* y = reinterpret_cast<double*>(ws + w.off_y);
  double* gmax = reinterpret_cast<double*>(ws + w.off_gmax);
  uint8_t* act = ws + w.off_act;
  int32_t* rows = reinterpret_cast<int32_t*>(ws + w.off_rows);
  int32_t* count = reinterpret_cast<int32_t*>(ws + w.off_count);
  const size_t blk = (size_t)kLuB * kLuB;
  // The decoupled modes (unit diagonal, zero row and column, lambda = 0)
  // drop out: the factorisation runs on the coupled block only, reached
  // through the row map and with its columns moved to the front of each
  // row.  The host learns the coupled count (one synchronisation).
  KALDO_LAUNCH("bte_flags", bte_flags, dim3((unsigned)((n_all + 255) / 256)), dim3(256), 0, st,
               n_all, omega, gamma0, gmax, nu_min_thz, act);
  KALDO_LAUNCH("bte_compact_index", bte_compact_index, dim3(1), dim3(1024), 0, st, n_all, act,
               rows, count);
  int32_t n_coupled = 0;
  KALDO_HIP(hipMemcpyAsync(&n_coupled, count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  KALDO_HIP(hipStreamSynchronize(st));
  const long n = n_coupled;
  const dim3 g3all((unsigned)((3 * n_all + 255) / 256));
  KALDO_LAUNCH("bte_zero", bte_zero, g3all, dim3(256), 0, st, (size_t)(3 * n_all), lambda);
  if (n > 0) {
    const MatRows A{matrix, rows, n_all};
    KALDO_LAUNCH("bte_compact_cols", bte_compact_cols, dim3((unsigned)n), dim3(256), 0, st, n,
                 n_all, rows, matrix);
    const int nb = (int)((n + kLuB - 1) / kLuB);
    // Blocked right-looking LU in panels of kLuPanel blocks: the steps inside
    // a panel update only the panel's columns (every row below) and the
    // panel's rows (every column to the right); the rest of the trailing
    // matrix takes one rank-(64 kLuPanel) product per panel (lu_gemm).
    for (int k0 = 0; k0 < nb; k0 += kLuPanel) {
      const int k1 = std::min(nb, k0 + kLuPanel);
      for (int k = k0; k < k1; ++k) {
        KALDO_LAUNCH("lu_diag", lu_diag, dim3(1), dim3(256), 0, st, n, k, A, linv + k * blk,
                     uinv + k * blk, c->d_flags);
        const int m = nb - k - 1;
        if (m == 0) continue;
        KALDO_LAUNCH("lu_panels", lu_panels, dim3(2 * m), dim3(256), 0, st, n, nb, k, A,
                     linv + k * blk, uinv + k * blk);
        const int pw = k1 - k - 1;  // panel columns (and rows) still to factor
        if (pw > 0) {
          // the panel's columns, every row below k; then the panel's rows,
          // the columns past the panel
          const int nr = nb - k1 > 0 ? pw * (nb - k1) : 0;
          KALDO_LAUNCH("lu_update", lu_update, dim3((unsigned)(m * pw + nr)), dim3(256), 0, st, n,
                       k, k + 1, k + 1, pw, m * pw, k + 1, k1, nb - k1 > 0 ? nb - k1 : 1, A);
        }
      }
      if (k1 < nb) {
        const long r0 = (long)k1 * kLuB;
        const int ntl = (int)((n - r0 + kLgT - 1) / kLgT);
        KALDO_LAUNCH("lu_gemm", lu_gemm, dim3((unsigned)(ntl * ntl)), dim3(256), 0, st, n, r0,
                     (long)k0 * kLuB, (k1 - k0) * kLuB, ntl, A);
      }
    }
    // the coupled right-hand sides, then forward: y = L^-1 b, the residual in
    // y2 (starting as b)
    double* r = reinterpret_cast<double*>(ws + w.off_y2);
    const dim3 g3((unsigned)((3 * n + 255) / 256));
    KALDO_LAUNCH("bte_gather3", bte_gather3, g3, dim3(256), 0, st, n, rows, rhs, r);
    for (int k = 0; k < nb; ++k)
      KALDO_LAUNCH("lu_step", lu_step<true>, dim3(nb - k), dim3(256), 0, st, n, k, linv + k * blk,
                   A, y, r);
    // backward: lambda = U^-1 y, the residual in y2 (starting as y)
    KALDO_LAUNCH("bte_copy3", bte_copy3, g3, dim3(256), 0, st, n, y, r);
    for (int k = nb - 1; k >= 0; --k)
      KALDO_LAUNCH("lu_step", lu_step<false>, dim3(k + 1), dim3(256), 0, st, n, k, uinv + k * blk,
                   A, lam_c, r);
    KALDO_LAUNCH("bte_scatter3", bte_scatter3, g3, dim3(256), 0, st, n, rows, lam_c, lambda);
  }
  const double scale = kKappaUnit / ((double)nq * c->volume);
  KALDO_LAUNCH("bte_kappa", bte_kappa, dim3(1), dim3(1024), 0, st, n_all, omega, vel, lambda, gamma0,
               gmax, kHbar / (kKb * temperature), nu_min_thz, scale, kappa);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_bte_iterate(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                                 const double* vel, const double* gamma0, double temperature,
                                 double nu_min_thz, const double* matrix, int32_t n_iterations,
                                 double tolerance, void* workspace, size_t workspace_bytes,
                                 double* lambda, double* kappa, int32_t* iterations,
                                 void* stream) {
  long nq = 0;
  int rc = check_common(c, mesh, temperature, &nq);
  if (rc) return rc;
  KALDO_REQUIRE(matrix && lambda && kappa, "kaldo_bte_iterate: NULL argument");
  KALDO_REQUIRE(n_iterations >= 0 && std::isfinite(tolerance) && tolerance >= 0,
                "kaldo_bte_iterate: bad n_iterations or tolerance");
  const BteWs w = bte_ws(c, nq);
  hipStream_t st = static_cast<hipStream_t>(stream);
  rc = bte_solve_common(c, mesh, omega, vel, gamma0, temperature, nu_min_thz, workspace,
                        workspace_bytes, w, nq, st);
  if (rc) return rc;
  auto* ws = static_cast<unsigned char*>(workspace);
  const long n = nq * c->nb3;
  double* rhs = reinterpret_cast<double*>(ws + w.off_rhs);
  double* y = reinterpret_cast<double*>(ws + w.off_y);
  double* gmax = reinterpret_cast<double*>(ws + w.off_gmax);
  double* kap_ws = reinterpret_cast<double*>(ws + w.off_kappa);
  const double scale = kKappaUnit / ((double)nq * c->volume);
  const double ikt = kHbar / (kKb * temperature);
  const dim3 g1((unsigned)((n + 255) / 256));
  KALDO_LAUNCH("bte_sc_init", bte_sc_init, g1, dim3(256), 0, st, n, rhs, gamma0, lambda);
  KALDO_LAUNCH("bte_kappa", bte_kappa, dim3(1), dim3(1024), 0, st, n, omega, vel, lambda, gamma0,
               gmax, ikt, nu_min_thz, scale, kap_ws);
  double kh[9];
  KALDO_HIP(hipMemcpyAsync(kh, kap_ws, sizeof(kh), hipMemcpyDeviceToHost, st));
  KALDO_HIP(hipStreamSynchronize(st));
  double k_prev = (kh[0] + kh[4] + kh[8]) / 3.0;
  int it = 0;
  bool conv = false;
  while (it < n_iterations) {
    KALDO_LAUNCH("bte_gemv", bte_gemv, dim3((unsigned)n), dim3(256), 0, st, n, matrix, lambda, y);
    KALDO_LAUNCH("bte_sc_update", bte_sc_update, g1, dim3(256), 0, st, n, rhs, gamma0, omega, gmax,
                 nu_min_thz, y, lambda);
    KALDO_LAUNCH("bte_kappa", bte_kappa, dim3(1), dim3(1024), 0, st, n, omega, vel, lambda, gamma0,
                 gmax, ikt, nu_min_thz, scale, kap_ws);
    KALDO_HIP(hipMemcpyAsync(kh, kap_ws, sizeof(kh), hipMemcpyDeviceToHost, st));
    KALDO_HIP(hipStreamSynchronize(st));
    ++it;
    const double k_new = (kh[0] + kh[4] + kh[8]) / 3.0;
    const bool stop = std::fabs(k_new - k_prev) <= tolerance * std::fabs(k_prev);
    k_prev = k_new;
    if (stop) {
      conv = true;
      break;
    }
  }
  KALDO_HIP(hipMemcpyAsync(kappa, kap_ws, sizeof(kh), hipMemcpyDeviceToDevice, st));
  KALDO_HIP(hipStreamSynchronize(st));
  if (iterations) *iterations = it;
  if (!conv || !std::isfinite(k_prev)) {
    set_error("kaldo_bte_iterate: no convergence within n_iterations (the iteration contracts only "
              "when the off-diagonal part is small against the diagonal); kappa is the last iterate's");
    return KALDO_ENUMERIC;
  }
  return KALDO_OK;
}
