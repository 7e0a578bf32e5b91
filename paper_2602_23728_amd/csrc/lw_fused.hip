// Fused crystal linewidth kernel: one workgroup per q-point.
//
// Paper: Eq. phi3_proj (projection on three Bloch eigenvectors), Eq. gamma
// with its Delta terms, Eq. broadening (only pairs with |x| < 2 sigma are
// projected, as the paper's implementation does), Eq. bose.
//
// Work of one workgroup (q fixed, all branches s at once):
//  1. A~_q (the FC3 COO contracted on its home-cell index with eta(q), with
//     the phase e^{+i q.R''} folded in) built in FP64 and stored in LDS in an
//     atom-block layout [block (jb, kb, d)][beta gamma][s].
//  2. The (q1, s') candidates are swept in chunks, one per thread: for every
//     s'' and s the FP64 energy cut |x+-| < 2 sigma+- of the oracle, with
//     x+ = (w + w1) - w2, x- = (w - w1) - w2, decides; the passing
//     (q1, s, s', s'') are compacted in a fixed order (block-wide exclusive
//     scan) into an LDS queue together with their FP64 weight.
//  3. When the queue is full (and at the end) every thread projects queue
//     entries: V = sum_blocks e^{-i q1.R_d} sum_{beta,gamma}
//     A~[blk][beta gamma][s] eta_{3jb+beta}(q1,s') eta_{3kb+gamma}(q2,s''),
//     in the contraction type T, and adds w |V|^2 (FP64) to its per-branch sum.
//  4. A fixed-order tree reduction over the workgroup gives Gamma(q, s).
// Every order above depends on the inputs only, so results are bitwise
// reproducible.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "common.h"
#include "lw_common.h"

namespace kaldo {

constexpr int kFusedThreads = 256;
constexpr int kFusedCap = 2048;

// Waves per SIMD the register allocation targets: four for the small FP32
// cells (measured: the latency of the gathers needs the extra wave), the
// compiler's choice otherwise.
template <int NB, typename T>
constexpr int fused_waves_per_eu() {
  return (NB <= 2 && sizeof(T) == 4) ? 4 : 1;
}

template <int NB, typename T>
__global__ __launch_bounds__(kFusedThreads)
__attribute__((amdgpu_waves_per_eu(fused_waves_per_eu<NB, T>()))) void lw_fused(
    LwParams p, int n_rep, const int32_t* __restrict__ rep, const double* __restrict__ omega,
    const double* __restrict__ vel, const double* __restrict__ occ,
    const uint8_t* __restrict__ phys, const uint8_t* __restrict__ sel,
    const int32_t* __restrict__ phys_list, const int32_t* __restrict__ n_phys_ptr,
    const double* __restrict__ evec, const typename Cx<T>::type* __restrict__ etaT,
    const typename Cx<T>::type* __restrict__ phase_tab, const int32_t* __restrict__ t_ptr,
    const int32_t* __restrict__ t_i, const int32_t* __restrict__ t_l2,
    const double* __restrict__ t_coef, const int32_t* __restrict__ e_blk,
    const int32_t* __restrict__ e_bg, const int32_t* __restrict__ blk_d,
    const int32_t* __restrict__ pair_ptr, double scale, double* __restrict__ gamma) {
  constexpr int NB3 = 3 * NB;
  constexpr int BS = kFusedThreads;
  constexpr int CAP = kFusedCap;
  using C = typename Cx<T>::type;
  extern __shared__ double2 smem[];
  C* at = reinterpret_cast<C*>(smem);  // [n_blk][9][NB3]
  __shared__ int rq_q1[CAP];
  __shared__ int rq_code[CAP];
  __shared__ int wave_tot[BS / 64];
  __shared__ double2 phq[64];
  __shared__ double wq64[NB3];
  __shared__ double red[BS];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int q = blockIdx.x;
  const int N0 = p.N[0], N1 = p.N[1], N2 = p.N[2];
  const int a0 = q / (N1 * N2), a1 = (q / N2) % N1, a2 = q % N2;

  float wqf[NB3];
  float wq_abs_max = 0.0f;
  unsigned live = 0, any_sel = 0;
#pragma unroll
  for (int s = 0; s < NB3; ++s) {
    const double w = omega[q * NB3 + s];
    wqf[s] = (float)w;
    wq_abs_max = fmaxf(wq_abs_max, fabsf((float)w));
    const bool ph = phys[q * NB3 + s], se = sel[q * NB3 + s];
    live |= (ph && se) ? (1u << s) : 0u;
    any_sel |= se ? (1u << s) : 0u;
  }
  if (live == 0) {
    if (tid < NB3 && (any_sel >> tid & 1u)) gamma[q * NB3 + tid] = 0.0;
    return;
  }
  if (tid < NB3) wq64[tid] = omega[q * NB3 + tid];

  // 1. A~_q in LDS
  for (int l = tid; l < n_rep; l += BS) {
    const int32_t* r = rep + 3 * l;
    int m0 = ((a0 * r[0]) % N0 + N0) % N0, m1 = ((a1 * r[1]) % N1 + N1) % N1,
        m2 = ((a2 * r[2]) % N2 + N2) % N2;
    double f = (double)m0 / N0 + (double)m1 / N1 + (double)m2 / N2;
    double sn, cs;
    sincospi(2.0 * f, &sn, &cs);
    phq[l] = make_double2(cs, sn);
  }
  const int n_at = p.n_blk * 9 * NB3;
  for (int k = tid; k < n_at; k += BS) at[k] = Cx<T>::make((T)0, (T)0);
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
    at[(e_blk[e] * 9 + e_bg[e]) * NB3 + s] = Cx<T>::make((T)re, (T)im);
  }
  __syncthreads();

  double acc[NB3];
#pragma unroll
  for (int s = 0; s < NB3; ++s) acc[s] = 0.0;

  // 3. projection of queue entries [0, n)
  auto process = [&](int n) {
    for (int r = tid; r < n; r += BS) {
      const int q1 = rq_q1[r];
      const int code = rq_code[r];
      const int s = code & 255, s1 = (code >> 8) & 255, s2 = code >> 16;
      const int b0 = q1 / (N1 * N2), b1 = (q1 / N2) % N1, b2 = q1 % N2;
      const int c0 = ((-a0 - b0) % N0 + N0) % N0, c1 = ((-a1 - b1) % N1 + N1) % N1,
                c2 = ((-a2 - b2) % N2 + N2) % N2;
      const int q2 = (c0 * N1 + c1) * N2 + c2;
      // FP64 weight of the entry (here, where every lane has an entry)
      const int m1 = q1 * NB3 + s1, m2 = q2 * NB3 + s2;
      double sp, sm;
      widths(p, vel, m1, m2, sp, sm);
      const double w = pair_weight(p, wq64[s], omega[m1], omega[m2], occ[m1], occ[m2], sp, sm);
      C x[NB3], y[NB3];
      const C* xs = etaT + ((size_t)q1 * NB3 + s1) * NB3;
      const C* ys = etaT + ((size_t)q2 * NB3 + s2) * NB3;
#pragma unroll
      for (int j = 0; j < NB3; ++j) {
        x[j] = xs[j];
        y[j] = ys[j];
      }
      const C* ph = phase_tab + (size_t)q1 * p.n_d;
      T vr = 0, vi = 0;
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
          const int b_lo = pair_ptr[jb * NB + kb], b_hi = pair_ptr[jb * NB + kb + 1];
          if (b_lo == b_hi) continue;
          C z[9];
#pragma unroll
          for (int be = 0; be < 3; ++be)
#pragma unroll
            for (int ga = 0; ga < 3; ++ga) {
              const C u = x[3 * jb + be], v = y[3 * kb + ga];
              z[be * 3 + ga] = Cx<T>::make(u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x);
            }
          for (int blk = b_lo; blk < b_hi; ++blk) {
            const C* ab = at + (size_t)blk * 9 * NB3 + s;
            T ur = 0, ui = 0;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
              const C a = ab[k * NB3];
              ur += a.x * z[k].x - a.y * z[k].y;
              ui += a.x * z[k].y + a.y * z[k].x;
            }
            const C f = ph[blk_d[blk]];
            vr += f.x * ur - f.y * ui;
            vi += f.x * ui + f.y * ur;
          }
        }
      }
      const double c = w * ((double)vr * (double)vr + (double)vi * (double)vi);
#pragma unroll
      for (int k = 0; k < NB3; ++k) acc[k] += (k == s) ? c : 0.0;
    }
  };

  // 2. sweep of the physical (q1, s') candidates
  int fill = 0;
  const int n_items = *n_phys_ptr;
  for (int base = 0; base < n_items; base += BS) {
    const int item = base + tid;
    unsigned bits[NB3];
#pragma unroll
    for (int k = 0; k < NB3; ++k) bits[k] = 0;
    int count = 0;
    int q1 = 0, s1 = 0, q2 = 0;
    if (item < n_items) {
      const int m1 = phys_list[item];
      q1 = m1 / NB3;
      s1 = m1 % NB3;
      const int b0 = q1 / (N1 * N2), b1 = (q1 / N2) % N1, b2 = q1 % N2;
      const int c0 = ((-a0 - b0) % N0 + N0) % N0, c1 = ((-a1 - b1) % N1 + N1) % N1,
                c2 = ((-a2 - b2) % N2 + N2) % N2;
      q2 = (c0 * N1 + c1) * N2 + c2;
      const double w1 = omega[m1];
      const double* v1 = vel + 3 * (size_t)m1;
#pragma unroll
      for (int s2 = 0; s2 < NB3; ++s2) {
        const int m2 = q2 * NB3 + s2;
        if (!phys[m2]) continue;
        const double w2 = omega[m2];
        double s2p, s2m, Sp, Sm;
        widths2(p, v1, vel + 3 * (size_t)m2, s2p, s2m, Sp, Sm);
        const float scl = wq_abs_max + fabsf((float)w1) + fabsf((float)w2);
        const Band bp = make_band(s2p, scl), bm = make_band(s2m, scl);
        const float cp = (float)(w1 - w2), cm = (float)(-w1 - w2);
        // certain passes and the ambiguous band for all branches first
        // (branch-free); the exact FP64 test only for the rare band members
        unsigned b = 0, amb_p = 0, amb_m = 0;
#pragma unroll
        for (int s = 0; s < NB3; ++s) {
          const float ap = fabsf(wqf[s] + cp), am = fabsf(wqf[s] + cm);
          b |= ((ap < bp.lo) || (am < bm.lo)) ? (1u << s) : 0u;
          amb_p |= (ap < bp.hi) ? (1u << s) : 0u;
          amb_m |= (am < bm.hi) ? (1u << s) : 0u;
        }
        unsigned amb = (amb_p | amb_m) & ~b & live;
        while (amb) {
          const int s = __ffs(amb) - 1;
          amb &= amb - 1;
          const bool pass = ((amb_p >> s & 1u) && exact_pass(p, wq64[s], w1, w2, Sp, Sm, true)) ||
                            ((amb_m >> s & 1u) && exact_pass(p, wq64[s], w1, w2, Sp, Sm, false));
          b |= pass ? (1u << s) : 0u;
        }
        b &= live;
        bits[s2] = b;
        count += __popc(b);
      }
    }
    // block-wide exclusive scan of count (fixed order)
    int incl = count;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wave_tot[wv] = incl;
    __syncthreads();
    int wave_off = 0, total = 0;
#pragma unroll
    for (int k = 0; k < BS / 64; ++k) {
      const int t = wave_tot[k];
      wave_off += (k < wv) ? t : 0;
      total += t;
    }
    const int my_off = wave_off + incl - count;
    __syncthreads();
    int written = 0;
    while (written < total) {
      const int take = min(CAP - fill, total - written);
      if (count > 0 && my_off < written + take && my_off + count > written) {
        int rank = my_off;
#pragma unroll
        for (int s2 = 0; s2 < NB3; ++s2) {
          unsigned b = bits[s2];
          while (b) {
            const int s = __ffs(b) - 1;
            b &= b - 1;
            if (rank >= written && rank < written + take) {
              const int slot = fill + rank - written;
              rq_q1[slot] = q1;
              rq_code[slot] = s | (s1 << 8) | (s2 << 16);
            }
            ++rank;
          }
        }
      }
      fill += take;
      written += take;
      __syncthreads();
      if (fill == CAP) {
        process(fill);
        fill = 0;
        __syncthreads();
      }
    }
  }
  process(fill);

  // 4. fixed-order reduction per branch
#pragma unroll
  for (int s = 0; s < NB3; ++s) {
    __syncthreads();
    red[tid] = acc[s];
    __syncthreads();
    for (int w = BS / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0 && (any_sel >> s & 1u))
      gamma[q * NB3 + s] = (live >> s & 1u) ? scale * red[0] : 0.0;
  }
}

// Deterministic compaction of the physical modes: list[k] = k-th mode with
// phys[m] != 0, *count = their number.  One workgroup.
__global__ __launch_bounds__(1024) void lw_compact_phys(int n_modes, const uint8_t* __restrict__ phys,
                                                        int32_t* __restrict__ list,
                                                        int32_t* __restrict__ count) {
  __shared__ int wave_tot[16];
  __shared__ int carry;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n_modes; base += 1024) {
    const int m = base + tid;
    const int f = (m < n_modes && phys[m]) ? 1 : 0;
    int incl = f;
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wave_tot[wv] = incl;
    __syncthreads();
    int off = carry, tot = 0;
    for (int k = 0; k < 16; ++k) {
      off += (k < wv) ? wave_tot[k] : 0;
      tot += wave_tot[k];
    }
    if (f) list[off + incl - 1] = m;
    __syncthreads();
    if (tid == 0) carry += tot;
    __syncthreads();
  }
  if (tid == 0) *count = carry;
}

// eta rounded to T and transposed to [q][mode][component].
template <typename T>
__global__ void lw_eta_transpose(long nq, int nb3, const double* __restrict__ evec,
                                 typename Cx<T>::type* __restrict__ etaT) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nq * nb3 * nb3) return;
  const int j = k % nb3, s = (k / nb3) % nb3;
  const long q = k / ((long)nb3 * nb3);
  const size_t src = ((q * nb3 + j) * nb3 + s) * 2;
  etaT[k] = Cx<T>::make((T)evec[src], (T)evec[src + 1]);
}

size_t fused_lds_bytes(const kaldo_crystal* c, int prec) {
  const size_t cs = prec == KALDO_FP64 ? 16 : 8;
  return (size_t)c->bloch.n_blk * 9 * c->nb3 * cs;
}

bool fused_supported(const kaldo_crystal* c, int prec) {
  if (c->nb < 1 || c->nb > 5 || c->n_rep > 64) return false;
  if (const char* f = std::getenv("KALDO_FORCE_GENERIC"))
    if (f[0] == '1') return false;
  int dev = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return false;
  // dynamic LDS plus the static queue / scan / reduction buffers
  const size_t stat = kFusedCap * 8 + kFusedThreads * 8 + 64 * 16 + 64;
  return fused_lds_bytes(c, prec) + stat <= (size_t)lds_max;
}

template <typename T>
int launch_fused(const kaldo_crystal* c, const LwParams& p, const double* omega, const double* vel,
                 const double* occ, const uint8_t* phys, const uint8_t* sel, const double* evec,
                 typename Cx<T>::type* eta, typename Cx<T>::type* phase_tab, int32_t* phys_list,
                 double scale, double* gamma, hipStream_t st) {
  const int nq = p.nq;
  const int n_modes = nq * c->nb3;
  const long ne = (long)n_modes * c->nb3;
  KALDO_LAUNCH("lw_eta_transpose", lw_eta_transpose<T>, dim3((ne + 255) / 256), dim3(256), 0, st,
               (long)nq, c->nb3, evec, eta);
  KALDO_LAUNCH("lw_compact_phys", lw_compact_phys, dim3(1), dim3(1024), 0, st, n_modes, phys,
               phys_list + 1, phys_list);
  const long nph = (long)nq * std::max(1, p.n_d);
  KALDO_LAUNCH("lw_phase_table", lw_phase_table<T>, dim3((nph + 255) / 256), dim3(256), 0, st, nq,
               p.n_d, p.N[0], p.N[1], p.N[2], c->bloch.dvec, phase_tab);
  const size_t lds = fused_lds_bytes(c, sizeof(T) == 8 ? KALDO_FP64 : KALDO_FP32);
  const Fc3Bloch& b = c->bloch;
#define KALDO_FUSED_CASE(NBV)                                                                  \
  case NBV:                                                                                    \
    KALDO_LAUNCH("lw_fused", (lw_fused<NBV, T>), dim3(nq), dim3(kFusedThreads), lds, st, p,    \
                 c->n_rep, c->d_rep, omega, vel, occ, phys, sel, phys_list + 1, phys_list, evec, \
                 eta, phase_tab, b.t_ptr,                                                    \
                 b.t_i, b.t_l2, b.t_coef, b.e_blk, b.e_bg, b.blk_d, b.pair_ptr, scale, gamma);  \
    break;
  switch (c->nb) {
    KALDO_FUSED_CASE(1)
    KALDO_FUSED_CASE(2)
    KALDO_FUSED_CASE(3)
    KALDO_FUSED_CASE(4)
    KALDO_FUSED_CASE(5)
    default:
      set_error("lw_fused: unsupported basis size");
      return KALDO_EUNSUPPORTED;
  }
#undef KALDO_FUSED_CASE
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

template int launch_fused<float>(const kaldo_crystal*, const LwParams&, const double*,
                                 const double*, const double*, const uint8_t*, const uint8_t*,
                                 const double*, float2*, float2*, int32_t*, double, double*,
                                 hipStream_t);
template int launch_fused<double>(const kaldo_crystal*, const LwParams&, const double*,
                                  const double*, const double*, const uint8_t*, const uint8_t*,
                                  const double*, double2*, double2*, int32_t*, double, double*,
                                  hipStream_t);

}  // namespace kaldo
