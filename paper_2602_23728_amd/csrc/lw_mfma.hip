// Crystal linewidths with the dense per-(q, q1) eigenvector contractions on
// the matrix cores (cells with up to 16 branches, zero-padded to 16).
//
// Paper: Eq. phi3_proj evaluated as in its "Computational Implementation":
// the home-cell contraction with eta(q) first (A~_q, in LDS), then for every
// partner q1 and branch s the two dense products
//     T_s = B_s eta(q2),   V_s = eta(q1)^T T_s,
//     B_s[jc][kc] = sum_d e^{-i q1.R_d} A~_q[d][jc][kc][s],
// followed by Eq. gamma / Eq. broadening / Eq. bose for all (s', s'') in FP64.
//
// A complex 16x16x16 product is two real products with the complex parts
// stacked along K (K = 32):  Re C = [Re A | -Im A][Re B ; Im B] and
// Im C = [Im A | Re A][Re B ; Im B].
//   FP32 form:  v_mfma_f32_16x16x4_f32, 8 per real product.
//   BF16x3:     v_mfma_f32_16x16x32_bf16 on x = hi + lo splits,
//               hi*hi + hi*lo + lo*hi per real product, FP32 accumulation.
// One workgroup per q (8 waves sharing A~_q in LDS, two per SIMD); each wave
// takes its own q1 values.  With Phi3 symmetric in its last two slots the
// tile of the mirrored partner (q2, q1) is V^T, so only q1 <_lex q2 is swept
// (q1 == q2 once) and each candidate carries the terms of both orderings.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "common.h"
#include "lw_common.h"

namespace kaldo {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;

constexpr int kMfmaWaves = 8;
constexpr int kMfmaThreads = 64 * kMfmaWaves;
constexpr int kMfmaMaxBlocks = 128;  // atom blocks (jb, kb, d) of the FC3 tables
constexpr int kCandCap = 2 * 64;     // a full batch plus one row's worth

// Order LDS traffic between the lanes of one wave (no workgroup barrier:
// the waves of a workgroup run different numbers of q1 iterations).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Complex K index of element i of a lane's operand fragment (g = lane / 16):
//   FP32 16x16x4, 8 MFMAs over the stacked K = 32: MFMA t reads stacked
//     k = 4 t + g, i.e. complex column kc = 4 (t % 4) + g, part t / 4.
//   BF16 16x16x32: element i reads stacked k = 8 g + i, i.e. complex column
//   kc = 8 (g % 2) + i, part g / 2.
// The second product V = eta1^T T takes its K order from the accumulator
// layout of T instead (lane (n, g) holds T rows 4 g + r, r < 4): FP32 MFMA t
// pairs K slot g with jc = 4 g + t % 4 (part t / 4), BF16 element i with
// jc = 4 g + i % 4 (part i / 4), so T goes from registers straight into the
// next product; eta1's fragments follow the same order.

template <bool SPLIT>
__global__ __launch_bounds__(kMfmaThreads) void lw_mfma(
    LwParams p, int n_rep, const int32_t* __restrict__ rep,
    const double* __restrict__ omega, const double* __restrict__ vel,
    const double* __restrict__ occ, const uint8_t* __restrict__ phys,
    const uint8_t* __restrict__ sel, const double* __restrict__ evec,
    const float2* __restrict__ phase_tab, const int32_t* __restrict__ t_ptr,
    const int32_t* __restrict__ t_i, const int32_t* __restrict__ t_l2,
    const double* __restrict__ t_coef, const int32_t* __restrict__ e_blk,
    const int32_t* __restrict__ e_bg, const int32_t* __restrict__ blk_d,
    const int4* __restrict__ bwork, double scale, double* __restrict__ gamma) {
  const int NB3 = p.nb3;
  extern __shared__ double2 smem[];
  float2* at = reinterpret_cast<float2*>(smem);  // [n_blk][9][NB3]
  __shared__ float2 bsc[kMfmaWaves][16 * 17];         // per-wave B_s tile [row jc][col kc]
  __shared__ float2 phb[kMfmaWaves][kMfmaMaxBlocks];  // per-wave e^{-i q1.R_d(blk)} per block
  __shared__ int cq_code[kMfmaWaves][kCandCap];       // per-wave near-shell candidates of the
  __shared__ double cq_v2[kMfmaWaves][kCandCap];      //   current partner: s | s' << 8 | s'' << 16, |V|^2
  __shared__ double md[kMfmaWaves][2][16][5];         // per-wave (w, n, v) of the q1 and q2 modes
  __shared__ double2 phq[64];
  __shared__ double wq64[16];
  __shared__ double red[kMfmaThreads];
  double acc[16];  // this thread's per-branch sums (registers)

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int q = blockIdx.x;
  const int N0 = p.N[0], N1 = p.N[1], N2 = p.N[2];
  const int a0 = q / (N1 * N2), a1 = (q / N2) % N1, a2 = q % N2;

  unsigned live = 0, any_sel = 0;
  float wq_abs_max = 0.0f;
  for (int s = 0; s < NB3; ++s) {
    const bool ph = phys[q * NB3 + s], se = sel[q * NB3 + s];
    live |= (ph && se) ? (1u << s) : 0u;
    any_sel |= se ? (1u << s) : 0u;
    wq_abs_max = fmaxf(wq_abs_max, fabsf((float)omega[q * NB3 + s]));
  }
  if (live == 0) {
    if (tid < NB3 && (any_sel >> tid & 1u)) gamma[q * NB3 + tid] = 0.0;
    return;
  }
  if (tid < NB3) wq64[tid] = omega[q * NB3 + tid];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int k = tid; k < kMfmaWaves * 16 * 17; k += kMfmaThreads) (&bsc[0][0])[k] = make_float2(0.f, 0.f);
  for (int l = tid; l < n_rep; l += kMfmaThreads) {
    const int32_t* r = rep + 3 * l;
    int m0 = ((a0 * r[0]) % N0 + N0) % N0, m1 = ((a1 * r[1]) % N1 + N1) % N1,
        m2 = ((a2 * r[2]) % N2 + N2) % N2;
    double f = (double)m0 / N0 + (double)m1 / N1 + (double)m2 / N2;
    double sn, cs;
    sincospi(2.0 * f, &sn, &cs);
    phq[l] = make_double2(cs, sn);
  }
  const int n_at = p.n_blk * 9 * NB3;
  for (int k = tid; k < n_at; k += kMfmaThreads) at[k] = make_float2(0.f, 0.f);
  __syncthreads();
  for (int k = tid; k < p.n_e * NB3; k += kMfmaThreads) {
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
    at[(e_blk[e] * 9 + e_bg[e]) * NB3 + s] = make_float2((float)re, (float)im);
  }
  __syncthreads();

  // entries of a lane's operand fragments
  constexpr int NF = SPLIT ? 8 : 4;
  auto kc_of = [&](int i) { return SPLIT ? 8 * (lg & 1) + i : 4 * i + lg; };
  // this lane's share of every B_s tile (fixed for the whole kernel)
  // packed as pos | lo << 9 | hi << 17 | bg << 25 (pos < 272, block indices
  // <= 128, bg < 9), -1 for no item
  int wk[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int4 w = bwork[k * 64 + lane];
    wk[k] = w.x < 0 ? -1 : (w.x | (w.y << 9) | (w.z << 17) | (w.w << 25));
  }

  // Exact FP64 cut and weight of queued candidates, one per lane, in queue
  // order, from the partner's mode data staged in LDS (the queue only ever
  // holds candidates of the current partner); the contribution goes to this
  // lane's sum of the candidate's branch.
  int n_cand = 0;  // wave-uniform
  auto resolve = [&](int dbl) {
    for (int base = 0; base < n_cand; base += 64) {
      const int e = base + lane;
      if (e < n_cand) {
        const int code = cq_code[wv][e];
        const int cs_ = code & 255, cs1 = (code >> 8) & 255, cs2 = (code >> 16) & 255;
        const double* d1 = md[wv][0][cs1];
        const double* d2 = md[wv][1][cs2];
        double sp, sm;
        widths_v(p, d1 + 2, d2 + 2, sp, sm);
        double wt = pair_weight(p, wq64[cs_], d1[0], d2[0], d1[1], d2[1], sp, sm);
        // the mirrored ordering: same |V|^2 and widths, its own cut
        if (dbl) wt += pair_weight(p, wq64[cs_], d2[0], d1[0], d2[1], d1[1], sp, sm);
        const double c = wt * cq_v2[wv][e];
        // register accumulators need a static index: add to the selected one
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] += (k == cs_) ? c : 0.0;
      }
    }
    n_cand = 0;
    wave_sync();
  };

  const Partners prt(p.half != 0, a0, a1, a2, N0, N1, N2);
  for (int pi = wv; pi < prt.n; pi += kMfmaWaves) {
    int b0, b1, b2;
    const int dbl = prt.get(pi, N1, N2, b0, b1, b2);  // wave-uniform
    const int q1 = (b0 * N1 + b1) * N2 + b2;
    const int c0 = ((-a0 - b0) % N0 + N0) % N0, c1 = ((-a1 - b1) % N1 + N1) % N1,
              c2 = ((-a2 - b2) % N2 + N2) % N2;
    const int q2 = (c0 * N1 + c1) * N2 + c2;
    wave_sync();
    for (int blk = lane; blk < p.n_blk; blk += 64)
      phb[wv][blk] = phase_tab[(size_t)q1 * p.n_d + blk_d[blk]];
    if ((lane & 15) < NB3 && lane < 32) {
      const int m = (lane < 16 ? q1 : q2) * NB3 + (lane & 15);
      double* d = md[wv][lane >> 4][lane & 15];
      d[0] = omega[m];
      d[1] = occ[m];
      d[2] = vel[3 * (size_t)m];
      d[3] = vel[3 * (size_t)m + 1];
      d[4] = vel[3 * (size_t)m + 2];
    }
    wave_sync();
    // eta(q2)[kc][s''] as the B operand of T = B_s eta2 (column n = lr)
    // and eta(q1)[jc][s'] (jc = 4 lg + i) as A = eta1^T (row m = lr) of
    // V = eta1^T T.
    float2 e2[NF], e1[4];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int k = kc_of(i);
      e2[i] = make_float2(0.f, 0.f);
      if (k < NB3 && lr < NB3) {
        const size_t o2 = (((size_t)q2 * NB3 + k) * NB3 + lr) * 2;
        if constexpr (SPLIT) {
          // B' stacks Re eta2 over Im eta2: lane groups 0, 1 take the real
          // part, 2, 3 the imaginary one.  The lane loads only its own
          // component; a run-time choice between the two halves of a
          // register pair would send the whole array to scratch memory.
          e2[i].x = (float)evec[o2 + (lg < 2 ? 0 : 1)];
        } else {
          e2[i] = make_float2((float)evec[o2], (float)evec[o2 + 1]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * lg + i;
      e1[i] = make_float2(0.f, 0.f);
      if (k < NB3 && lr < NB3) {
        const size_t o1 = (((size_t)q1 * NB3 + k) * NB3 + lr) * 2;
        e1[i] = make_float2((float)evec[o1], (float)evec[o1 + 1]);
      }
    }
    // this lane's epilogue pairs: s' = 4 lg + r, s'' = lr.  Only the FP32
    // pre-classification data stay in registers; the exact FP64 decision and
    // weight reload their inputs (rare: candidates near the energy shell).
    const int s2 = lr;
    unsigned pr_ok = 0;
    float bhi_p[4], bhi_m[4], cpv[4], cmv[4];
    const bool s2_ok = s2 < NB3 && phys[q2 * NB3 + s2];
    const double w2 = s2_ok ? omega[q2 * NB3 + s2] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int s1 = 4 * lg + r;
      bhi_p[r] = bhi_m[r] = cpv[r] = cmv[r] = 0.f;
      if (s2_ok && s1 < NB3 && phys[q1 * NB3 + s1]) {
        pr_ok |= 1u << r;
        const int m1 = q1 * NB3 + s1;
        const double w1 = omega[m1];
        double s2p, s2m, Sp, Sm;
        widths2(p, vel + 3 * (size_t)m1, vel + 3 * (size_t)(q2 * NB3 + s2), s2p, s2m, Sp, Sm);
        const float scl = wq_abs_max + fabsf((float)w1) + fabsf((float)w2);
        const float d = 4e-7f * scl + 1e-9f;
        bhi_p[r] = 2.0f * band_sqrt((float)s2p) * (1.0f + 1e-6f) + d;
        bhi_m[r] = 2.0f * band_sqrt((float)s2m) * (1.0f + 1e-6f) + d;
        // with the mirrored ordering, |w + cp| and |w - cp| share the edge
        // bhi_p, and for w >= 0 the smaller is |w - |cp|| (bitwise in FP32):
        // one test covers both
        cpv[r] = dbl ? -fabsf((float)(w1 - w2)) : (float)(w1 - w2);
        cmv[r] = (float)(-w1 - w2);
      }
    }
    // operand fragments of eta that do not depend on s
    bf16x8 e2h, e2l, e1ah, e1al, e1bh, e1bl;  // BF16 form
    float e2f[8], e1af[8], e1bf[8];            // FP32 form
    if constexpr (SPLIT) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        // B' = [Re eta2 ; Im eta2]; A'(eta1^T) = [Re | -Im], A'' = [Im | Re]
        const float b = e2[i].x;
        const float a1 = (i < 4) ? e1[i & 3].x : -e1[i & 3].y;
        const float a2 = (i < 4) ? e1[i & 3].y : e1[i & 3].x;
        e2h[i] = (__bf16)b;
        e2l[i] = (__bf16)(b - (float)e2h[i]);
        e1ah[i] = (__bf16)a1;
        e1al[i] = (__bf16)(a1 - (float)e1ah[i]);
        e1bh[i] = (__bf16)a2;
        e1bl[i] = (__bf16)(a2 - (float)e1bh[i]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int i = t & 3;
        e2f[t] = (t < 4) ? e2[i].x : e2[i].y;
        e1af[t] = (t < 4) ? e1[i].x : -e1[i].y;
        e1bf[t] = (t < 4) ? e1[i].y : e1[i].x;
      }
    }
#pragma unroll 1
    for (int s = 0; s < NB3; ++s) {
      if (!(live >> s & 1u)) continue;  // uniform
      // B_s tile built cooperatively into LDS, then read as operand fragments
      float2* Bt = bsc[wv];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (wk[k] < 0) continue;
        const int pos = wk[k] & 511, lo = (wk[k] >> 9) & 255, end = (wk[k] >> 17) & 255,
                  bg = (wk[k] >> 25) & 15;
        float2 v = make_float2(0.f, 0.f);
        const int stride = 9 * NB3;
        const float2* ap = at + (lo * 9 + bg) * NB3 + s;
        int blk = lo;
        // four blocks per round: their LDS loads are issued together
        for (; blk + 4 <= end; blk += 4, ap += 4 * stride) {
          float2 a[4], f[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            a[j] = ap[j * stride];
            f[j] = phb[wv][blk + j];
          }
          // complex multiply-adds as fused multiply-adds into v (four per
          // product instead of two multiplies, two fused and two adds)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            v.x = fmaf(f[j].x, a[j].x, v.x);
            v.x = fmaf(-f[j].y, a[j].y, v.x);
            v.y = fmaf(f[j].x, a[j].y, v.y);
            v.y = fmaf(f[j].y, a[j].x, v.y);
          }
        }
        for (; blk < end; ++blk, ap += stride) {
          const float2 a = *ap;
          const float2 f = phb[wv][blk];
          v.x = fmaf(f.x, a.x, v.x);
          v.x = fmaf(-f.y, a.y, v.x);
          v.y = fmaf(f.x, a.y, v.y);
          v.y = fmaf(f.y, a.x, v.y);
        }
        Bt[pos] = v;
      }
      wave_sync();
      float2 bv[NF];
#pragma unroll
      for (int i = 0; i < NF; ++i) bv[i] = Bt[lr * 17 + kc_of(i)];
      f4 tr = {0, 0, 0, 0}, ti = {0, 0, 0, 0};
      if constexpr (SPLIT) {
        bf16x8 a1h, a1l, a2h, a2l;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float a1 = (lg < 2) ? bv[i].x : -bv[i].y;
          const float a2 = (lg < 2) ? bv[i].y : bv[i].x;
          a1h[i] = (__bf16)a1;
          a1l[i] = (__bf16)(a1 - (float)a1h[i]);
          a2h[i] = (__bf16)a2;
          a2l[i] = (__bf16)(a2 - (float)a2h[i]);
        }
        tr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1l, e2h, tr, 0, 0, 0);
        tr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1h, e2l, tr, 0, 0, 0);
        tr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1h, e2h, tr, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2l, e2h, ti, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2h, e2l, ti, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2h, e2h, ti, 0, 0, 0);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int i = t & 3;
          const float a1 = (t < 4) ? bv[i].x : -bv[i].y;
          const float a2 = (t < 4) ? bv[i].y : bv[i].x;
          tr = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, e2f[t], tr, 0, 0, 0);
          ti = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, e2f[t], ti, 0, 0, 0);
        }
      }
      // T (rows 4 lg + r of column lr, in registers) is the B operand of V
      f4 vr = {0, 0, 0, 0}, vi = {0, 0, 0, 0};
      if constexpr (SPLIT) {
        bf16x8 th, tl;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float b = (i < 4) ? tr[i & 3] : ti[i & 3];
          th[i] = (__bf16)b;
          tl[i] = (__bf16)(b - (float)th[i]);
        }
        vr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e1al, th, vr, 0, 0, 0);
        vr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e1ah, tl, vr, 0, 0, 0);
        vr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e1ah, th, vr, 0, 0, 0);
        vi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e1bl, th, vi, 0, 0, 0);
        vi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e1bh, tl, vi, 0, 0, 0);
        vi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(e1bh, th, vi, 0, 0, 0);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float b = (t < 4) ? tr[t & 3] : ti[t & 3];
          vr = __builtin_amdgcn_mfma_f32_16x16x4f32(e1af[t], b, vr, 0, 0, 0);
          vi = __builtin_amdgcn_mfma_f32_16x16x4f32(e1bf[t], b, vi, 0, 0, 0);
        }
      }
      // epilogue: V[s' = 4 lg + r][s'' = lr].  The FP32 pre-classification
      // drops candidates certainly outside the cut; the rest are queued with
      // their |V|^2 for the exact FP64 decision and weight.
      const float wsf = (float)wq64[s];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        bool near = false;
        if (pr_ok >> r & 1u) {
          // coalescence of either ordering, or decay (w > 0: s is live)
          near = fabsf(wsf + cpv[r]) < bhi_p[r] || fabsf(wsf + cmv[r]) < bhi_m[r];
        }
        const unsigned long long mask = __ballot(near);
        if (near) {
          const unsigned lo = (unsigned)mask, hi = (unsigned)(mask >> 32);
          const int off = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
          const int slot = n_cand + off;
          cq_code[wv][slot] = s | ((4 * lg + r) << 8) | (s2 << 16);
          cq_v2[wv][slot] = (double)vr[r] * (double)vr[r] + (double)vi[r] * (double)vi[r];
        }
        n_cand += __popcll(mask);
        if (n_cand >= 64) {
          wave_sync();
          resolve(dbl);
        }
      }
      wave_sync();
    }
    resolve(dbl);  // the queue never carries candidates past their partner
  }
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    if (s >= NB3) break;
    __syncthreads();
    red[tid] = acc[s];
    __syncthreads();
    for (int w = kMfmaThreads / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0 && (any_sel >> s & 1u))
      gamma[q * NB3 + s] = (live >> s & 1u) ? scale * red[0] : 0.0;
  }
}

bool mfma_supported(const kaldo_crystal* c) {
  if (c->nb3 > 16 || c->n_rep > 64 || c->bloch.n_blk > kMfmaMaxBlocks) return false;
  int dev = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return false;
  const size_t dyn = (size_t)c->bloch.n_blk * 9 * c->nb3 * 8;
  const size_t stat = kMfmaWaves * 16 * 17 * 8 + kMfmaWaves * kMfmaMaxBlocks * 8 +
                      kMfmaWaves * kCandCap * 12 + kMfmaWaves * 2 * 16 * 5 * 8 + 64 * 16 + 16 * 8 + kMfmaThreads * 8;
  return dyn + stat <= (size_t)lds_max;
}

int launch_mfma(const kaldo_crystal* c, const LwParams& p, bool split, const double* omega,
                const double* vel, const double* occ, const uint8_t* phys, const uint8_t* sel,
                const double* evec, float2* phase_tab, double scale, double* gamma,
                hipStream_t st) {
  const int nq = p.nq;
  const long nph = (long)nq * std::max(1, p.n_d);
  KALDO_LAUNCH("lw_phase_table", lw_phase_table<float>, dim3((nph + 255) / 256), dim3(256), 0, st,
               nq, p.n_d, p.N[0], p.N[1], p.N[2], c->bloch.dvec, phase_tab);
  const size_t lds = (size_t)c->bloch.n_blk * 9 * c->nb3 * 8;
  const Fc3Bloch& b = c->bloch;
  if (split)
    KALDO_LAUNCH("lw_mfma_bf16x3", lw_mfma<true>, dim3(nq), dim3(kMfmaThreads), lds, st, p,
                 c->n_rep, c->d_rep, omega, vel, occ, phys, sel, evec, phase_tab, b.t_ptr, b.t_i,
                 b.t_l2, b.t_coef, b.e_blk, b.e_bg, b.blk_d, b.bwork, scale, gamma);
  else
    KALDO_LAUNCH("lw_mfma_fp32", lw_mfma<false>, dim3(nq), dim3(kMfmaThreads), lds, st, p,
                 c->n_rep, c->d_rep, omega, vel, occ, phys, sel, evec, phase_tab, b.t_ptr, b.t_i,
                 b.t_l2, b.t_coef, b.e_blk, b.e_bg, b.blk_d, b.bwork, scale, gamma);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

}  // namespace kaldo
