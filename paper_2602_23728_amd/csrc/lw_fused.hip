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
//  2. The (q1, s') candidates are swept in rounds, one per thread (the FP64
//     pass: a partner q1 per thread, swept once per s'): for every
//     s'' and s the energy cut |x+-| < 2 sigma+- of the oracle, with
//     x+ = (w + w1) - w2, x- = (w - w1) - w2, decides (pre-classified in FP32
//     against a conservative band from the FP32 mode copies; band members
//     take the FP64 test); the passing (q1, q2, s, s', s'') are compacted in
//     a fixed order (block-wide exclusive scan) into an LDS queue.  When Phi3
//     is symmetric in its last two slots the ordered pair (q1 s', q2 s'')
//     and its mirror (q2 s'', q1 s') have the same V, so only q1 <_lex q2 is
//     swept (and q1 == q2 once) and an entry carries the terms of both
//     orderings, each with its own cut.
//  3. When the queue is full (and at the end) every thread projects queue
//     entries: V = sum_blocks e^{-i q1.R_d} sum_{beta,gamma}
//     A~[blk][beta gamma][s] eta_{3jb+beta}(q1,s') eta_{3kb+gamma}(q2,s''),
//     in the contraction type T, and adds w |V|^2 (FP64) to its per-branch sum.
//  4. A fixed-order tree reduction over the workgroup gives this work
//     item's partial sum; lw_fused_finish adds the chunks of a q in order.
// A workgroup takes one work item (q, chunk): a live q and a contiguous
// share of its sweep, so a subset of a few hundred q-points still fills the
// device.
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
// cells, three for the small FP64 cells (measured: the latency of the gathers
// needs the extra waves; 20.8 -> 18.5 ms on the diamond 24^3 mesh in FP64
// with 14 spilled registers, while four waves spill 53), the compiler's
// choice otherwise.
template <int NB, typename T>
constexpr int fused_waves_per_eu() {
  return (NB <= 2 && sizeof(T) == 4) ? 4 : (NB <= 2 ? 3 : 1);
}

// Whether the sweep runs in blocks of partners, each swept once per branch
// s' (the FP64 linewidth pass), or in rounds of (q1, s') items (the FP32
// forms, and the temperature cache's count and record passes, which must
// split their work items alike; its FP64 record pass spills 19 registers
// with partner blocks against 2).
template <typename T, int MODE>
constexpr bool fused_partner_blocks() {
  return sizeof(T) == 8 && MODE == kModeGamma;
}

// Gamma of the selected modes: the chunk sums of their q in chunk order.
__global__ void lw_fused_finish(int n_modes, int nb3, const uint8_t* __restrict__ phys,
                                const uint8_t* __restrict__ sel, const int32_t* __restrict__ idx_of_q,
                                int n_chunk, const double* __restrict__ part, double scale,
                                double* __restrict__ gamma) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_modes || !sel[m]) return;
  const int q = m / nb3, s = m - q * nb3, k = idx_of_q[q];
  if (!phys[m] || k < 0) {
    gamma[m] = 0.0;
    return;
  }
  double acc = 0.0;
  for (int c = 0; c < n_chunk; ++c) acc += part[((size_t)k * kFusedMaxChunks + c) * nb3 + s];
  gamma[m] = scale * acc;
}

// MODE (FusedMode): kModeGamma sums the linewidth terms into `part`;
// kModeCount runs only the sweep's cut decisions and writes the number of
// passing entries per branch of this work item to tc.count; kModeRecord
// re-runs the same decisions, projects the passing entries and stores each
// one's temperature-independent factors at a fixed place of its mode's row:
// the row start, plus the counts of the earlier chunks, plus its rank among
// the chunk's entries of that branch in queue order.
template <int NB, typename T, int MODE = kModeGamma>
__global__ __launch_bounds__(kFusedThreads)
__attribute__((amdgpu_waves_per_eu(fused_waves_per_eu<NB, T>()))) void lw_fused(
    LwParams p, int n_rep, const int32_t* __restrict__ rep, const double* __restrict__ omega,
    const double* __restrict__ vel, const float4* __restrict__ modef, const double* __restrict__ occ,
    const double2* __restrict__ mrec, const uint8_t* __restrict__ phys,
    const uint8_t* __restrict__ sel, const double* __restrict__ evec,
    const typename Cx<T>::type* __restrict__ etaT,
    const typename Cx<T>::type* __restrict__ phase_tab, const int32_t* __restrict__ t_ptr,
    const int32_t* __restrict__ t_i, const int32_t* __restrict__ t_l2,
    const double* __restrict__ t_coef, const int32_t* __restrict__ e_blk,
    const int32_t* __restrict__ e_bg, const int32_t* __restrict__ blk_d,
    const int32_t* __restrict__ pair_ptr, const int32_t* __restrict__ live_list,
    const int32_t* __restrict__ n_live_ptr, int n_chunk, double* __restrict__ part, TcOut tc) {
  constexpr int NB3 = 3 * NB;
  constexpr int BS = kFusedThreads;
  constexpr int CAP = kFusedCap;
  constexpr bool kRecord = MODE == kModeRecord;
  constexpr int NPK = (NB3 + 1) / 2;  // branch counters packed two per int (16 bits each)
  using C = typename Cx<T>::type;
  extern __shared__ double2 smem[];
  C* at = reinterpret_cast<C*>(smem);  // [n_blk][9][NB3]
  __shared__ int rq_q1[CAP];
  __shared__ int rq_q2[CAP];
  __shared__ int rq_code[CAP];
  __shared__ int rq_dst[kRecord ? CAP : 1];  // rank of the entry within its branch's share
  __shared__ long long rbase[NB3];           // where this work item's entries of a branch start
  __shared__ long long rlim[NB3];            // and how many the count pass found
  __shared__ int wave_tot[BS / 64];
  __shared__ int wave_tot_s[BS / 64][NPK];
  __shared__ double2 phq[64];
  __shared__ double wq64[NB3];
  __shared__ float wqs[NB3];  // FP32 frequencies of q, indexed per candidate
  __shared__ double red[BS];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int N0 = p.N[0], N1 = p.N[1], N2 = p.N[2];
  // workgroup = one (live q, chunk) work item; the grid may hold more
  // workgroups than there are items
  const int n_work = *n_live_ptr * n_chunk;
  {
    const int wk = blockIdx.x;
    if (wk >= n_work) return;
    const int kq = wk / n_chunk, chunk = wk - kq * n_chunk;
    const int q = live_list[kq];
    const int a0 = q / (N1 * N2), a1 = (q / N2) % N1, a2 = q % N2;

    float wqf[NB3];
    float wq_abs_max = 0.0f;
    unsigned live = 0;
#pragma unroll
    for (int s = 0; s < NB3; ++s) {
      const double w = omega[q * NB3 + s];
      wqf[s] = (float)w;
      wq_abs_max = fmaxf(wq_abs_max, fabsf((float)w));
      live |= (phys[q * NB3 + s] && sel[q * NB3 + s]) ? (1u << s) : 0u;
    }
    // FP32 frequencies of the live branches, +inf for the others (they then
    // fail every band test of the sweep)
    float wql[NB3];
#pragma unroll
    for (int s = 0; s < NB3; ++s) wql[s] = (live >> s & 1u) ? wqf[s] : __builtin_inff();
    if (tid < NB3) wq64[tid] = omega[q * NB3 + tid];
    if (tid < NB3) wqs[tid] = (float)omega[q * NB3 + tid];
    if constexpr (kRecord) {
      if (tid < NB3) {
        long long b = tc.row_ptr[q * NB3 + tid];
        for (int c = 0; c < chunk; ++c) b += tc.count[((size_t)kq * kFusedMaxChunks + c) * NB3 + tid];
        rbase[tid] = b;
        rlim[tid] = tc.count[((size_t)kq * kFusedMaxChunks + chunk) * NB3 + tid];
      }
    }

    // 1. A~_q in LDS (the count pass projects nothing)
    if constexpr (MODE == kModeCount) __syncthreads();
    if constexpr (MODE != kModeCount) {
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
    }

    double acc[NB3];
    int cnt[NB3];  // count pass: this thread's passing entries per branch
    int run[NB3];  // record pass: entries of each branch in the rounds before
#pragma unroll
    for (int s = 0; s < NB3; ++s) {
      acc[s] = 0.0;
      cnt[s] = 0;
      run[s] = 0;
    }

    // 3. projection of queue entries [0, n)
    auto process = [&](int n) {
      for (int r = tid; r < n; r += BS) {
        const int q1 = rq_q1[r], q2 = rq_q2[r];
        const int code = rq_code[r];
        const int s = code & 255, s1 = (code >> 8) & 255, s2 = (code >> 16) & 255, dbl = code >> 24;
        // FP64 weight of the entry (here, where every lane has an entry),
        // from the partners' packed (w, n, v) records
        const int m1 = q1 * NB3 + s1, m2 = q2 * NB3 + s2;
        const double2 a1 = mrec[3 * (size_t)m1], b1 = mrec[3 * (size_t)m1 + 1],
                      c1 = mrec[3 * (size_t)m1 + 2];
        const double2 a2 = mrec[3 * (size_t)m2], b2 = mrec[3 * (size_t)m2 + 1],
                      c2 = mrec[3 * (size_t)m2 + 2];
        const double w1 = a1.x, n1 = a1.y, w2 = a2.x, n2 = a2.y;
        double sp, sm;
        {
          const double v1[3] = {b1.x, b1.y, c1.x}, v2[3] = {b2.x, b2.y, c2.x};
          widths_v(p, v1, v2, sp, sm);
        }
        double w = 0.0;
        if constexpr (MODE == kModeGamma) {
          w = pair_weight(p, wq64[s], w1, w2, n1, n2, sp, sm);
          // the mirrored ordering: same widths (|v1 +- v2| are symmetric), its own cut
          if (dbl) w += pair_weight(p, wq64[s], w2, w1, n2, n1, sp, sm);
        }
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
        // V = sum_blk f_blk sum_beta x_beta (sum_gamma A~[blk][beta gamma] y_gamma):
        // complex multiply-adds as chains of fused multiply-adds into the
        // accumulators (four per product; the written form a.x b.x - a.y b.y
        // costs a multiply, a fused one and an add per component), and no
        // x (x) y table (nine complex values a block would have to keep or
        // recompute)
        // One block's term f_blk x_jb^T A~_blk y_kb into (vr, vi).  The FP64
        // Gamma pass loads the three values of a row of the block together
        // and fetches each block's phase one block ahead, so that the
        // latencies fall under arithmetic; the FP32 form and the record pass
        // have no registers left for either.
        constexpr bool kAhead = sizeof(T) == 8 && MODE == kModeGamma;
        auto block_term = [&](const C* ab, const C f, int jb, int kb) {
          T ur = 0, ui = 0;
#pragma unroll
          for (int be = 0; be < 3; ++be) {
            C a[3];
            if constexpr (kAhead) {
#pragma unroll
              for (int ga = 0; ga < 3; ++ga) a[ga] = ab[(be * 3 + ga) * NB3];
            }
            T tr = 0, ti = 0;
#pragma unroll
            for (int ga = 0; ga < 3; ++ga) {
              if constexpr (!kAhead) a[ga] = ab[(be * 3 + ga) * NB3];
              const C v = y[3 * kb + ga];
              tr = fma(a[ga].x, v.x, tr);
              tr = fma(-a[ga].y, v.y, tr);
              ti = fma(a[ga].x, v.y, ti);
              ti = fma(a[ga].y, v.x, ti);
            }
            const C u = x[3 * jb + be];
            ur = fma(u.x, tr, ur);
            ur = fma(-u.y, ti, ur);
            ui = fma(u.x, ti, ui);
            ui = fma(u.y, tr, ui);
          }
          vr = fma(f.x, ur, vr);
          vr = fma(-f.y, ui, vr);
          vi = fma(f.x, ui, vi);
          vi = fma(f.y, ur, vi);
        };
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
#pragma unroll
          for (int kb = 0; kb < NB; ++kb) {
            const int b_lo = pair_ptr[jb * NB + kb], b_hi = pair_ptr[jb * NB + kb + 1];
            if constexpr (kAhead) {
              C f_next = Cx<T>::make((T)0, (T)0);
              if (b_lo < b_hi) f_next = ph[blk_d[b_lo]];
              for (int blk = b_lo; blk < b_hi; ++blk) {
                const C f = f_next;
                if (blk + 1 < b_hi) f_next = ph[blk_d[blk + 1]];
                block_term(at + (size_t)blk * 9 * NB3 + s, f, jb, kb);
              }
            } else {
              for (int blk = b_lo; blk < b_hi; ++blk)
                block_term(at + (size_t)blk * 9 * NB3 + s, ph[blk_d[blk]], jb, kb);
            }
          }
        }
        const double v2 = (double)vr * (double)vr + (double)vi * (double)vi;
        if constexpr (kRecord) {
          // a+ (n1 - n2) + 1/2 a- (n1 + n2 + 1) of this ordering plus, when
          // the entry stands for both, the mirrored one's a+r (n2 - n1) +
          // 1/2 a-r (n1 + n2 + 1): stored as c (n1 - n2) + d (n1 + n2 + 1)
          double ap, am;
          pair_factors(p, wq64[s], w1, w2, sp, sm, ap, am);
          if (dbl) {
            double apr, amr;
            pair_factors(p, wq64[s], w2, w1, sp, sm, apr, amr);
            ap -= apr;
            am += amr;
          }
          // both passes take the same decisions, so the rank is below the
          // count; a write outside this work item's share is refused
          if (rq_dst[r] < rlim[s]) {
            const long long dst = rbase[s] + rq_dst[r];
            tc.pairs[dst] = make_uint2((unsigned)m1, (unsigned)m2);
            tc.factors[dst] = make_double2(v2 * ap, 0.5 * (v2 * am));
          } else {
            raise_flag(tc.flags, kFlagCache);
          }
        } else {
          const double c = w * v2;
#pragma unroll
          for (int k = 0; k < NB3; ++k) acc[k] += (k == s) ? c : 0.0;
        }
      }
    };

    // 2. sweep of the (q1, s') candidates (modes below the floor fail every
    // comparison through their NaN frequency)
    int fill = 0;
    const Partners prt(p.half != 0, a0, a1, a2, N0, N1, N2);
    // this work item's share: a contiguous range of whole sweep rounds.  The
    // FP64 linewidth pass (kBlk) sweeps blocks of BS partners: a thread
    // decodes its partner once per block (run-time divisions and range
    // tests, paid per wave whatever the number of lanes that need them) and
    // sweeps it once per branch s', a round being one (block, s') pair.  The
    // FP32 forms (four waves per SIMD) and the cache passes have no registers
    // for that and sweep (q1, s') items, a round being BS consecutive items.
    constexpr bool kBlk = fused_partner_blocks<T, MODE>();
    const int n_all = kBlk ? prt.n : prt.n * NB3;
    const int per = ((n_all + n_chunk - 1) / n_chunk + BS - 1) / BS * BS;
    const int i_lo = min(n_all, chunk * per), n_items = min(n_all, i_lo + per);
    for (int base = i_lo; base < n_items; base += BS) {
      const int item = base + tid;
      const bool have = item < n_items;
      int q1 = 0, q2_blk = 0, dbl = 0, s1_item = 0;
      if (have) {
        const int qi = kBlk ? item : item / NB3;
        s1_item = kBlk ? 0 : item - qi * NB3;
        int b0, b1, b2;
        dbl = prt.get(qi, N1, N2, b0, b1, b2);
        q1 = (b0 * N1 + b1) * N2 + b2;
        q2_blk = (wrap_sub(prt.h[0].t, b0, N0) * N1 + wrap_sub(prt.h[1].t, b1, N1)) * N2 +
             wrap_sub(prt.h[2].t, b2, N2);
      }
#pragma unroll 1
      for (int sr = 0; sr < (kBlk ? NB3 : 1); ++sr) {
        const int s1 = kBlk ? sr : s1_item;
        // q2 as seen by this round: an empty register barrier keeps the
        // compiler from hoisting the partner's per-branch addresses (six 64-bit
        // pointers of the rare exact path) out of the s' loop, where they spill
        int q2 = q2_blk;
        if constexpr (kBlk) asm volatile("" : "+v"(q2));
        unsigned bits[NB3];
#pragma unroll
        for (int k = 0; k < NB3; ++k) bits[k] = 0;
        int count = 0;
        if (have) {
          const int m1 = q1 * NB3 + s1;
          const float4 f1 = modef[m1];
          // the partner's mode copies one branch ahead, so that each load is
          // in flight while the previous branch is classified
          const float4* f2p = modef + (size_t)q2 * NB3;
          float4 f2n = f2p[0];
#pragma unroll
          for (int s2 = 0; s2 < NB3; ++s2) {
            const int m2 = q2 * NB3 + s2;
            // FP32 classification from the mode copies (a mode below the floor
            // carries a NaN frequency and fails every comparison)
            const float4 f2 = f2n;
            if (s2 + 1 < NB3) f2n = f2p[s2 + 1];
            float s2p, s2m, e_sig;
            widths2_f(p, f1, f2, s2p, s2m, e_sig);
            const float scl = wq_abs_max + fabsf(f1.w) + fabsf(f2.w);
            const Band bp = make_band_f(s2p, scl, e_sig), bm = make_band_f(s2m, scl, e_sig);
            const float cp = f1.w - f2.w, cm = -f1.w - f2.w;
            // The upper band edge for all branches first (branch-free): a
            // candidate is any process with |x| < hi.  The coalescence |x+| =
            // |w + cp| and that of the mirrored ordering, |w - cp| (= (w + w2) -
            // w1), share the edge bp.hi, and for w >= 0 the smaller of the two
            // is |w - |cp||, bitwise in FP32 (w + cp and w - cp round
            // monotonically); so one test per branch covers both, with cpe =
            // -|cp| on mirrored entries and cp otherwise.  The decay |x-| is the
            // same FP32 number for both orderings.  Live branches of q have w
            // >= 2 pi nu_min > 0; the others drop out through `live`.
            // The common path asks only whether any live branch is near: the
            // smallest |x| of each process over the branches against its edge
            // (a minimum is exact, so the answer is that of the per-branch
            // tests; a NaN x leaves the minimum at +inf or NaN, which fail).
            const float cpe = dbl ? -fabsf(cp) : cp;
            float xp[NB3], xm[NB3];
            float mp = __builtin_inff(), mm = __builtin_inff();
#pragma unroll
            for (int s = 0; s < NB3; ++s) {
              xp[s] = wql[s] + cpe;
              xm[s] = wql[s] + cm;
              mp = fminf(mp, fabsf(xp[s]));
              mm = fminf(mm, fabsf(xm[s]));
            }
            unsigned b = 0;
            if (mp < bp.hi || mm < bm.hi) {
              unsigned cand = 0;
#pragma unroll
              for (int s = 0; s < NB3; ++s)
                cand |= (fabsf(xp[s]) < bp.hi || fabsf(xm[s]) < bm.hi) ? (1u << s) : 0u;
              cand &= live;
              // the rare candidates: which process is near (as the tests above),
              // certain passes in FP32, the band members take the exact FP64 test
              unsigned amb = 0, amb_p = 0, amb_r = 0, amb_m = 0;
              for (unsigned c = cand; c; c &= c - 1) {
                const int s = __ffs(c) - 1;
                const float w = wqs[s];
                const float ap = fabsf(w + cp), ar = fabsf(w - cp), am = fabsf(w + cm);
                const bool hp = ap < bp.hi, hr = dbl && ar < bp.hi, hm = am < bm.hi;
                amb_p |= hp ? (1u << s) : 0u;
                amb_r |= hr ? (1u << s) : 0u;
                amb_m |= hm ? (1u << s) : 0u;
                const bool sure = (hp && ap < bp.lo) || (hm && am < bm.lo) || (hr && ar < bp.lo);
                b |= sure ? (1u << s) : 0u;
                amb |= sure ? 0u : (1u << s);
              }
              if (amb) {
                const double w1 = omega[m1], w2 = omega[m2];
                double s2p64, s2m64, Sp, Sm;
                widths2(p, vel + 3 * (size_t)m1, vel + 3 * (size_t)m2, s2p64, s2m64, Sp, Sm);
                while (amb) {
                  const int s = __ffs(amb) - 1;
                  amb &= amb - 1;
                  const bool bm_ = amb_m >> s & 1u;
                  bool pass = ((amb_p >> s & 1u) && exact_pass(p, wq64[s], w1, w2, Sp, Sm, true)) ||
                              (bm_ && exact_pass(p, wq64[s], w1, w2, Sp, Sm, false));
                  if (dbl && !pass)
                    pass = ((amb_r >> s & 1u) && exact_pass(p, wq64[s], w2, w1, Sp, Sm, true)) ||
                           (bm_ && exact_pass(p, wq64[s], w2, w1, Sp, Sm, false));
                  b |= pass ? (1u << s) : 0u;
                }
              }
            }
            b &= live;
            bits[s2] = b;
            count += __popc(b);
          }
        }
        if constexpr (MODE == kModeCount) {
#pragma unroll
          for (int s2 = 0; s2 < NB3; ++s2)
#pragma unroll
            for (int s = 0; s < NB3; ++s) cnt[s] += (int)((bits[s2] >> s) & 1u);
          continue;  // no queue: the round ends here (no barrier was passed)
        }
        // record pass: per-branch counts of this thread, packed two per int
        // (a round holds at most BS * NB3 < 2^16 entries of one branch)
        int pk[NPK], pk_incl[NPK];
        if constexpr (kRecord) {
#pragma unroll
          for (int k = 0; k < NPK; ++k) pk[k] = 0;
#pragma unroll
          for (int s2 = 0; s2 < NB3; ++s2)
#pragma unroll
            for (int s = 0; s < NB3; ++s) pk[s >> 1] += (int)((bits[s2] >> s) & 1u) << ((s & 1) * 16);
#pragma unroll
          for (int k = 0; k < NPK; ++k) {
            int v = pk[k];
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
              const int t = __shfl_up(v, off, 64);
              if (lane >= off) v += t;
            }
            pk_incl[k] = v;
            if (lane == 63) wave_tot_s[wv][k] = v;
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
        // record pass: this thread's first rank per branch within the round and
        // the round's total per branch
        int s_off[NB3], s_tot[NB3];
        if constexpr (kRecord) {
#pragma unroll
          for (int k = 0; k < NPK; ++k) {
            int off = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < BS / 64; ++w) {
              const int t = wave_tot_s[w][k];
              off += (w < wv) ? t : 0;
              tot += t;
            }
            const int ex = off + pk_incl[k] - pk[k];
            s_off[2 * k] = ex & 0xffff;
            s_tot[2 * k] = tot & 0xffff;
            if (2 * k + 1 < NB3) {
              s_off[2 * k + 1] = (int)((unsigned)ex >> 16);
              s_tot[2 * k + 1] = (int)((unsigned)tot >> 16);
            }
          }
        }
        __syncthreads();
        int written = 0;
        while (written < total) {
          const int take = min(CAP - fill, total - written);
          if (count > 0 && my_off < written + take && my_off + count > written) {
            int rank = my_off;
            if constexpr (kRecord) {
              // the order of the loop below (s'' ascending, then s ascending),
              // with static indices into the per-branch counters
              int loc[NB3];
#pragma unroll
              for (int s = 0; s < NB3; ++s) loc[s] = 0;
#pragma unroll
              for (int s2 = 0; s2 < NB3; ++s2) {
#pragma unroll
                for (int s = 0; s < NB3; ++s) {
                  if ((bits[s2] >> s) & 1u) {
                    if (rank >= written && rank < written + take) {
                      const int slot = fill + rank - written;
                      rq_q1[slot] = q1;
                      rq_q2[slot] = q2;
                      rq_code[slot] = s | (s1 << 8) | (s2 << 16) | (dbl << 24);
                      rq_dst[slot] = run[s] + s_off[s] + loc[s];
                    }
                    ++loc[s];
                    ++rank;
                  }
                }
              }
            } else {
#pragma unroll
              for (int s2 = 0; s2 < NB3; ++s2) {
                unsigned b = bits[s2];
                while (b) {
                  const int s = __ffs(b) - 1;
                  b &= b - 1;
                  if (rank >= written && rank < written + take) {
                    const int slot = fill + rank - written;
                    rq_q1[slot] = q1;
                    rq_q2[slot] = q2;
                    rq_code[slot] = s | (s1 << 8) | (s2 << 16) | (dbl << 24);
                  }
                  ++rank;
                }
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
        if constexpr (kRecord) {
#pragma unroll
          for (int s = 0; s < NB3; ++s) run[s] += s_tot[s];
        }
      }
    }

    if constexpr (MODE == kModeCount) {
      // 4c. entries per branch of this work item (integer sums: any order)
      __shared__ int cnt_red[BS / 64][NB3];
#pragma unroll
      for (int s = 0; s < NB3; ++s) {
        int v = cnt[s];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) cnt_red[wv][s] = v;
      }
      __syncthreads();
      if (tid < NB3) {
        long long t = 0;
#pragma unroll
        for (int w = 0; w < BS / 64; ++w) t += cnt_red[w][tid];
        tc.count[((size_t)kq * kFusedMaxChunks + chunk) * NB3 + tid] = t;
      }
      return;
    }
    process(fill);
    if constexpr (kRecord) return;

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
      if (tid == 0) part[((size_t)kq * kFusedMaxChunks + chunk) * NB3 + s] = red[0];
    }
  }
}

// Row pointers of the temperature cache: the entry count of mode (q, s) is
// the sum over its chunks (0 when q has no live mode), rows in mode order.
// One workgroup; each thread scans a contiguous run of modes, then one
// block-wide scan of the runs' sums places them.
__global__ __launch_bounds__(1024) void tc_rows(int n_modes, int nb3,
                                                const int32_t* __restrict__ idx_of_q, int n_chunk,
                                                const long long* __restrict__ count,
                                                long long* __restrict__ row_ptr) {
  __shared__ long long sums[1024];
  const int tid = threadIdx.x;
  const int per = (n_modes + 1023) / 1024;
  const int lo = min(n_modes, tid * per), hi = min(n_modes, lo + per);
  auto mode_count = [&](int m) -> long long {
    const int q = m / nb3, s = m - q * nb3, k = idx_of_q[q];
    if (k < 0) return 0;
    long long t = 0;
    for (int c = 0; c < n_chunk; ++c) t += count[((size_t)k * kFusedMaxChunks + c) * nb3 + s];
    return t;
  };
  long long own = 0;
  for (int m = lo; m < hi; ++m) own += mode_count(m);
  sums[tid] = own;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const long long v = tid >= off ? sums[tid - off] : 0;
    __syncthreads();
    sums[tid] += v;
    __syncthreads();
  }
  long long r = sums[tid] - own;
  for (int m = lo; m < hi; ++m) {
    row_ptr[m] = r;
    r += mode_count(m);
  }
  if (tid == 1023) row_ptr[n_modes] = sums[1023];
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

// Static LDS of the kernel besides the A~ tables: the queue, scan and
// reduction buffers, and for the cache's record pass the per-entry ranks.
static size_t fused_static_lds(bool record) {
  const size_t stat = kFusedCap * 12 + kFusedThreads * 8 + 64 * 16 + 64 + 4 * 8 * 4 + 16 * 8;
  return stat + (record ? kFusedCap * 4 : 0);
}

static bool fused_fits(const kaldo_crystal* c, int prec, bool record) {
  if (c->nb < 1 || c->nb > 5 || c->n_rep > 64) return false;
  int dev = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return false;
  return fused_lds_bytes(c, prec) + fused_static_lds(record) <= (size_t)lds_max;
}

bool fused_supported(const kaldo_crystal* c, int prec) {
  if (const char* f = std::getenv("KALDO_FORCE_GENERIC"))
    if (f[0] == '1') return false;
  return fused_fits(c, prec, false);
}
bool fused_record_supported(const kaldo_crystal* c, int prec) { return fused_fits(c, prec, true); }

// The fused launch of one mode: tables, live list, chunking and the kernel,
// then what the mode needs after it (the Gamma finish, or the cache's row
// pointers).  Count and record passes of one request see the same live list
// and chunk count, so they make the same cut decisions in the same order.
template <typename T, int MODE>
static int launch_fused_impl(const kaldo_crystal* c, const LwParams& p, const double* omega,
                             const double* vel, const float4* modef, const double* occ,
                             const double2* mrec, const uint8_t* phys, const uint8_t* sel,
                             const double* evec,
                             typename Cx<T>::type* eta, typename Cx<T>::type* phase_tab,
                             int32_t* qlist, double* part, int64_t n_subset, double scale,
                             double* gamma, TcOut tc, hipStream_t st) {
  const int nq = p.nq;
  const int n_modes = nq * c->nb3;
  const long ne = (long)n_modes * c->nb3;
  int32_t* live_list = qlist;
  int32_t* idx_of_q = qlist + nq;
  int32_t* n_live = qlist + 2 * nq;
  if (MODE != kModeCount) {
    KALDO_LAUNCH("lw_eta_transpose", lw_eta_transpose<T>, dim3((ne + 255) / 256), dim3(256), 0, st,
                 (long)nq, c->nb3, evec, eta);
    const long nph = (long)nq * std::max(1, p.n_d);
    KALDO_LAUNCH("lw_phase_table", lw_phase_table<T>, dim3((nph + 255) / 256), dim3(256), 0, st, nq,
                 p.n_d, p.N[0], p.N[1], p.N[2], c->bloch.dvec, phase_tab);
  }
  if (n_subset > 0)
    KALDO_LAUNCH("lw_live_q", lw_live_q<>, dim3(1), dim3(1024), 0, st, nq, c->nb3, phys, sel, live_list,
                 idx_of_q, n_live);
  else
    KALDO_LAUNCH("lw_all_q", lw_all_q<>, dim3((nq + 255) / 256), dim3(256), 0, st, nq, live_list,
                 idx_of_q, n_live);
  // the count pass builds no A~ tables: no dynamic LDS
  const size_t lds =
      MODE == kModeCount ? 0 : fused_lds_bytes(c, sizeof(T) == 8 ? KALDO_FP64 : KALDO_FP32);
  const Fc3Bloch& b = c->bloch;
  // Chunks per q from the number of live q-points the host can know of: at
  // most min(N_q, n_subset) (the grid covers that many), estimated as
  // n_subset / 3N_b (every branch of a q selected) when choosing the chunk
  // count, for about kWorkItems work items (four per resident workgroup on
  // a 256-CU device; a fixed count keeps the summation order, and so the
  // bits of Gamma, the same on every device).
  const long upper = n_subset > 0 ? std::min<long>(nq, n_subset) : nq;
  const long guess = n_subset > 0 ? std::max<long>(1, n_subset / c->nb3) : nq;
  // and no chunk shorter than one sweep round (a q sweeps about N_q / 2
  // partners, N_q 3N_b / 2 items)
  const long per_q = fused_partner_blocks<T, MODE>() ? (long)nq : (long)nq * c->nb3;
  const int max_chunks =
      (int)std::max<long>(1, std::min<long>(kFusedMaxChunks, per_q / (2 * kFusedThreads)));
  const int n_chunk =
      std::min(fused_chunks((int)std::min<long>(guess, 1l << 30), kWorkItems), max_chunks);
#define KALDO_FUSED_CASE(NBV)                                                                    \
  case NBV:                                                                                      \
    KALDO_LAUNCH("lw_fused", (lw_fused<NBV, T, MODE>), dim3((unsigned)(upper * n_chunk)),        \
                 dim3(kFusedThreads), lds, st, p, c->n_rep, c->d_rep, omega, vel, modef, occ,    \
                 mrec, phys, sel, evec, eta, phase_tab, b.t_ptr, b.t_i, b.t_l2, b.t_coef, b.e_blk, \
                 b.e_bg, b.blk_d, b.pair_ptr, live_list, n_live, n_chunk, part, tc);             \
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
  if (MODE == kModeGamma)
    KALDO_LAUNCH("lw_fused_finish", lw_fused_finish, dim3((n_modes + 255) / 256), dim3(256), 0, st,
                 n_modes, c->nb3, phys, sel, idx_of_q, n_chunk, part, scale, gamma);
  if (MODE == kModeCount)
    KALDO_LAUNCH("tc_rows", tc_rows, dim3(1), dim3(1024), 0, st, n_modes, c->nb3, idx_of_q, n_chunk,
                 tc.count, tc.row_ptr);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

template <typename T>
int launch_fused(const kaldo_crystal* c, const LwParams& p, const double* omega, const double* vel,
                 const float4* modef, const double* occ, const double2* mrec, const uint8_t* phys,
                 const uint8_t* sel, const double* evec, typename Cx<T>::type* eta,
                 typename Cx<T>::type* phase_tab, int32_t* qlist, double* part, int64_t n_subset,
                 double scale, double* gamma, hipStream_t st) {
  return launch_fused_impl<T, kModeGamma>(c, p, omega, vel, modef, occ, mrec, phys, sel, evec, eta,
                                          phase_tab, qlist, part, n_subset, scale, gamma, TcOut{},
                                          st);
}

template <typename T>
int launch_fused_cache(const kaldo_crystal* c, const LwParams& p, int mode, const double* omega,
                       const double* vel, const float4* modef, const double2* mrec,
                       const uint8_t* phys, const uint8_t* sel, const double* evec,
                       typename Cx<T>::type* eta, typename Cx<T>::type* phase_tab, int32_t* qlist,
                       int64_t n_subset, TcOut tc, hipStream_t st) {
  if (mode == kModeCount)
    return launch_fused_impl<T, kModeCount>(c, p, omega, vel, modef, nullptr, mrec, phys, sel, evec,
                                            eta, phase_tab, qlist, nullptr, n_subset, 0.0, nullptr,
                                            tc, st);
  return launch_fused_impl<T, kModeRecord>(c, p, omega, vel, modef, nullptr, mrec, phys, sel, evec,
                                           eta, phase_tab, qlist, nullptr, n_subset, 0.0, nullptr,
                                           tc, st);
}

template int launch_fused<float>(const kaldo_crystal*, const LwParams&, const double*,
                                 const double*, const float4*, const double*, const double2*,
                                 const uint8_t*, const uint8_t*, const double*, float2*, float2*,
                                 int32_t*, double*, int64_t, double, double*, hipStream_t);
template int launch_fused<double>(const kaldo_crystal*, const LwParams&, const double*,
                                  const double*, const float4*, const double*, const double2*,
                                  const uint8_t*, const uint8_t*, const double*, double2*, double2*,
                                  int32_t*, double*, int64_t, double, double*, hipStream_t);
template int launch_fused_cache<float>(const kaldo_crystal*, const LwParams&, int, const double*,
                                       const double*, const float4*, const double2*,
                                       const uint8_t*, const uint8_t*, const double*, float2*,
                                       float2*, int32_t*, int64_t, TcOut, hipStream_t);
template int launch_fused_cache<double>(const kaldo_crystal*, const LwParams&, int, const double*,
                                        const double*, const float4*, const double2*,
                                        const uint8_t*, const uint8_t*, const double*, double2*,
                                        double2*, int32_t*, int64_t, TcOut, hipStream_t);

}  // namespace kaldo
