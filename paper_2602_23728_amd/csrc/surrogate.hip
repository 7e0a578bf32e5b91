// Learned linewidth form: joint density of states, per-mode features, an MLP
// ensemble trained and evaluated by hand-written kernels, the disagreement
// gate with its calibration, and the irreducible-wedge map.
//
// The paper restricts the scattering calculation to the irreducible wedge and
// maps results back onto the full grid (overview of the 2.0 computational
// changes) and lists the phase space among its computed quantities ("Phonon
// Properties and Scattering"); it has no surrogate.  The network, its
// features and the gate are this library's own, built on the same energy
// cut, smearing and widths as the linewidths.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <vector>

#include "common.h"
#include "lw_common.h"

namespace kaldo {

constexpr int kMlpHidden = 64;
constexpr int kMlpDepth = 4;
constexpr int kMlpMaxIn = 32;
constexpr int kMlpMaxMembers = 16;
constexpr int kJdosThreads = 256;
constexpr int kTrainWaves = 8;
constexpr int kTrainThreads = 64 * kTrainWaves;
constexpr int kPredRows = 16;
constexpr int kGateMaxRows = 4096;
constexpr unsigned kSpinCap = 1u << 20;

// ----------------------------------------------------------------- JDOS
// Work item (live q, chunk): a share of the partner sweep of q.  Every
// unordered partner pair {q1, q2 = -q - q1} is visited once and contributes
// the terms of both orderings (the JDOS has no vertex, so this holds for any
// crystal): D+ gets g((w + w1) - w2) and g((w + w2) - w1), D- gets
// g((w - w1) - w2) and g((w - w2) - w1), each with its own exact FP64 cut.
// The sweep pre-classifies in FP32 (the band of the linewidths, so no term
// inside the cut is dropped) and queues candidates with a 4-bit term mask;
// the queue is evaluated densely (cut, smearing in FP64) and summed per
// branch in queue order; fixed-order reductions within the work item, then
// over the chunks of a q (jdos_finish).
constexpr int kJdosCap = 2048;

template <int NBM>  // branches held per thread: 3 N_b <= NBM
__global__ __launch_bounds__(kJdosThreads) void jdos_kernel(
    LwParams p, const double* __restrict__ omega, const double* __restrict__ vel,
    const float4* __restrict__ modef, const uint8_t* __restrict__ phys,
    const uint8_t* __restrict__ sel, const int32_t* __restrict__ live_list,
    const int32_t* __restrict__ n_live_ptr, int n_chunk, double* __restrict__ part) {
  constexpr int BS = kJdosThreads;
  __shared__ int rq_q1[kJdosCap];
  __shared__ int rq_code[kJdosCap];
  __shared__ int wave_tot[BS / 64];
  __shared__ double wq64[NBM];
  __shared__ double red[BS];
  const int NB3 = p.nb3;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wk = blockIdx.x;
  if (wk >= *n_live_ptr * n_chunk) return;
  const int kq = wk / n_chunk, chunk = wk - kq * n_chunk;
  const int q = live_list[kq];
  const int N0 = p.N[0], N1 = p.N[1], N2 = p.N[2];
  const int a0 = q / (N1 * N2), a1 = (q / N2) % N1, a2 = q % N2;
  unsigned live = 0;
  float wqf[NBM];
  float wq_abs_max = 0.0f;
#pragma unroll
  for (int s = 0; s < NBM; ++s) {
    const double w = s < NB3 ? omega[q * NB3 + s] : 0.0;
    wqf[s] = (float)w;
    wq_abs_max = fmaxf(wq_abs_max, fabsf(wqf[s]));
    if (s < NB3) live |= (phys[q * NB3 + s] && sel[q * NB3 + s]) ? 1u << s : 0u;
  }
  if (tid < NB3) wq64[tid] = omega[q * NB3 + tid];
  __syncthreads();

  double accp[NBM], accm[NBM];
#pragma unroll
  for (int s = 0; s < NBM; ++s) accp[s] = accm[s] = 0.0;

  // queue entries [0, n): exact cuts and smearing of the flagged terms
  auto process = [&](int n) {
    for (int r = tid; r < n; r += BS) {
      const int q1 = rq_q1[r], code = rq_code[r];
      const int s = code & 255, s1 = (code >> 8) & 255, s2 = (code >> 16) & 255, fl = code >> 24;
      const int b0 = q1 / (N1 * N2), b1 = (q1 / N2) % N1, b2 = q1 % N2;
      const int c0 = ((-a0 - b0) % N0 + N0) % N0, c1 = ((-a1 - b1) % N1 + N1) % N1,
                c2 = ((-a2 - b2) % N2 + N2) % N2;
      const int m1 = q1 * NB3 + s1, m2 = ((c0 * N1 + c1) * N2 + c2) * NB3 + s2;
      const double w = wq64[s], w1 = omega[m1], w2 = omega[m2];
      double sp, sm;
      widths(p, vel, m1, m2, sp, sm);
      double gp = 0.0, gm = 0.0;
      if (fl & 1) {
        const double x = (w + w1) - w2;
        if (fabs(x) < 2.0 * sp) gp += smear(p.shape, x, sp);
      }
      if (fl & 4) {
        const double x = (w + w2) - w1;
        if (fabs(x) < 2.0 * sp) gp += smear(p.shape, x, sp);
      }
      if (fl & 2) {
        const double x = (w - w1) - w2;
        if (fabs(x) < 2.0 * sm) gm += smear(p.shape, x, sm);
      }
      if (fl & 8) {
        const double x = (w - w2) - w1;
        if (fabs(x) < 2.0 * sm) gm += smear(p.shape, x, sm);
      }
#pragma unroll
      for (int k = 0; k < NBM; ++k) {
        accp[k] += (k == s) ? gp : 0.0;
        accm[k] += (k == s) ? gm : 0.0;
      }
    }
  };

  // sweep: this work item's share of the partner points, whole rounds
  const Partners prt(true, a0, a1, a2, N0, N1, N2);
  const int n_all = prt.n * NB3;
  const int per = ((n_all + n_chunk - 1) / n_chunk + BS - 1) / BS * BS;
  const int i_lo = min(n_all, chunk * per), i_hi = min(n_all, i_lo + per);
  int fill = 0;
  for (int base = i_lo; base < i_hi; base += BS) {
    const int item = base + tid;
    unsigned bpm[NBM], brr[NBM];  // per s'': D+ | D- << 16 of this ordering; D+ of the mirror
#pragma unroll
    for (int k = 0; k < NBM; ++k) bpm[k] = brr[k] = 0;
    int count = 0, q1 = 0, s1 = 0, dbl = 0;
    if (item < i_hi) {
      const int qi = item / NB3;
      s1 = item - qi * NB3;
      int b0, b1, b2;
      dbl = prt.get(qi, N1, N2, b0, b1, b2);
      q1 = (b0 * N1 + b1) * N2 + b2;
      const int q2 = (wrap_sub(prt.h[0].t, b0, N0) * N1 + wrap_sub(prt.h[1].t, b1, N1)) * N2 +
                     wrap_sub(prt.h[2].t, b2, N2);
      const float4 f1 = modef[q1 * NB3 + s1];
      const unsigned dmask = dbl ? ~0u : 0u;
      // the partner's mode copies (NaN frequency below the floor); up to 8
      // branches one branch ahead, each load in flight while the previous
      // branch is classified (with 16 the extra registers halve occupancy)
      const float4* f2p = modef + (size_t)q2 * NB3;
      float4 f2n = f2p[0];
#pragma unroll
      for (int s2 = 0; s2 < NBM; ++s2) {
        if (s2 >= NB3) break;
        float4 f2;
        if constexpr (NBM <= 8) {
          f2 = f2n;
          if (s2 + 1 < NB3) f2n = f2p[s2 + 1];
        } else {
          f2 = f2p[s2];
        }
        float s2p, s2m, e_sig;
        widths2_f(p, f1, f2, s2p, s2m, e_sig);
        const float scl = wq_abs_max + fabsf(f1.w) + fabsf(f2.w);
        const Band bp = make_band_f(s2p, scl, e_sig), bm = make_band_f(s2m, scl, e_sig);
        const float cp = f1.w - f2.w, cm = -f1.w - f2.w;
        unsigned mp = 0, mm = 0, mr = 0;
#pragma unroll
        for (int s = 0; s < NBM; ++s) {
          const float ap = fabsf(wqf[s] + cp), ar = fabsf(wqf[s] - cp), am = fabsf(wqf[s] + cm);
          mp |= (ap < bp.hi) ? (1u << s) : 0u;
          mr |= (ar < bp.hi) ? (1u << s) : 0u;
          mm |= (am < bm.hi) ? (1u << s) : 0u;
        }
        mp &= live;
        mm &= live;
        mr &= live & dmask;
        bpm[s2] = mp | (mm << 16);
        brr[s2] = mr;
        count += __popc(mp | mm | mr);
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
      const int take = min(kJdosCap - fill, total - written);
      if (count > 0 && my_off < written + take && my_off + count > written) {
        int rank = my_off;
#pragma unroll
        for (int s2 = 0; s2 < NBM; ++s2) {
          if (s2 >= NB3) break;
          const unsigned mp = bpm[s2] & 0xffffu, mm = bpm[s2] >> 16, mr = brr[s2];
          unsigned any = mp | mm | mr;
          while (any) {
            const int s = __ffs(any) - 1;
            any &= any - 1;
            if (rank >= written && rank < written + take) {
              const int fl = (mp >> s & 1u) | (mm >> s & 1u) << 1 | (mr >> s & 1u) << 2 |
                             ((mm >> s & 1u) & dbl) << 3;
              const int slot = fill + rank - written;
              rq_q1[slot] = q1;
              rq_code[slot] = s | (s1 << 8) | (s2 << 16) | (fl << 24);
            }
            ++rank;
          }
        }
      }
      fill += take;
      written += take;
      __syncthreads();
      if (fill == kJdosCap) {
        process(fill);
        fill = 0;
        __syncthreads();
      }
    }
  }
  process(fill);

  double* out = part + ((size_t)kq * kFusedMaxChunks + chunk) * 32;
#pragma unroll
  for (int s = 0; s < NBM; ++s) {
    if (s >= NB3) break;
    for (int which = 0; which < 2; ++which) {
      __syncthreads();
      red[tid] = which ? accm[s] : accp[s];
      __syncthreads();
      for (int w = BS / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
      }
      if (tid == 0) out[2 * s + which] = red[0];
    }
  }
}

// D+- of the selected modes: the chunk sums of their q in chunk order, / N_q;
// 0 below nu_min.
__global__ void jdos_finish(int n_modes, int nb3, int nq, const uint8_t* __restrict__ phys,
                            const uint8_t* __restrict__ sel, const int32_t* __restrict__ idx_of_q,
                            int n_chunk, const double* __restrict__ part,
                            double* __restrict__ dplus, double* __restrict__ dminus) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_modes || !sel[m]) return;
  const int q = m / nb3, s = m - q * nb3, k = idx_of_q[q];
  double sp = 0.0, sm = 0.0;
  if (phys[m] && k >= 0)
    for (int c = 0; c < n_chunk; ++c) {
      sp += part[((size_t)k * kFusedMaxChunks + c) * 32 + 2 * s];
      sm += part[((size_t)k * kFusedMaxChunks + c) * 32 + 2 * s + 1];
    }
  dplus[m] = phys[m] ? sp / nq : 0.0;
  dminus[m] = phys[m] ? sm / nq : 0.0;
}

// Flags and the FP32 (v, omega) mode copies of the sweep (omega NaN below
// nu_min, so that every comparison against such a mode fails).
__global__ void jdos_prepare(int n_modes, const double* __restrict__ omega,
                             const double* __restrict__ vel, double nu_min,
                             uint8_t* __restrict__ phys, uint8_t* __restrict__ sel,
                             float4* __restrict__ modef, int sel_all, int32_t* __restrict__ flags) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_modes) return;
  const double w = omega[m];
  const bool ph = (w / kTwoPi) >= nu_min;
  phys[m] = ph;
  sel[m] = sel_all ? 1 : 0;
  const double v0 = vel[3 * (size_t)m], v1 = vel[3 * (size_t)m + 1], v2 = vel[3 * (size_t)m + 2];
  modef[m] = make_float4((float)v0, (float)v1, (float)v2, ph ? (float)w : __builtin_nanf(""));
  if (!((w - w) + (v0 - v0) + (v1 - v1) + (v2 - v2) == 0.0)) raise_flag(flags, kFlagNonFinite);
  if (w < 0.0 && (-w / kTwoPi) >= nu_min) raise_flag(flags, kFlagImaginary);
}

__global__ void jdos_select(const int32_t* __restrict__ subset, long n, int n_modes,
                            uint8_t* __restrict__ sel, int32_t* __restrict__ flags) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int m = subset[k];
  if (m >= 0 && m < n_modes)
    sel[m] = 1;
  else
    raise_flag(flags, kFlagSubset);
}

// ----------------------------------------------------------------- features
// Row k (mode m = modes[k]): nu (THz), |v| (A/ps), one-hot branch (nb3), the
// ascending |components| of the shortest Cartesian image q + G (1/A), |q + G|,
// ln(1 + D+), ln(1 + D-).
__global__ void features_kernel(int nb3, int N0, int N1, int N2, double3 b0v, double3 b1v,
                                double3 b2v, const double* __restrict__ omega,
                                const double* __restrict__ vel, const double* __restrict__ dplus,
                                const double* __restrict__ dminus, const int32_t* __restrict__ modes,
                                int n, int n_feat, float* __restrict__ X) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int m = modes[k];
  const int q = m / nb3, s = m % nb3;
  const int n0 = q / (N1 * N2), n1 = (q / N2) % N1, n2 = q % N2;
  float* x = X + (size_t)k * n_feat;
  int f = 0;
  x[f++] = (float)(omega[m] / kTwoPi);
  const double* v = vel + 3 * (size_t)m;
  x[f++] = (float)sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int b = 0; b < nb3; ++b) x[f++] = (b == s) ? 1.0f : 0.0f;
  const double f0 = (double)n0 / N0, f1 = (double)n1 / N1, f2 = (double)n2 / N2;
  double best[3] = {0, 0, 0}, bl = 1e300;
  for (int i = -1; i <= 1; ++i)
    for (int j = -1; j <= 1; ++j)
      for (int l = -1; l <= 1; ++l) {
        const double c0 = f0 + i, c1 = f1 + j, c2 = f2 + l;
        const double qx = c0 * b0v.x + c1 * b1v.x + c2 * b2v.x;
        const double qy = c0 * b0v.y + c1 * b1v.y + c2 * b2v.y;
        const double qz = c0 * b0v.z + c1 * b1v.z + c2 * b2v.z;
        const double L = qx * qx + qy * qy + qz * qz;
        if (L < bl - 1e-12) {
          bl = L;
          best[0] = fabs(qx);
          best[1] = fabs(qy);
          best[2] = fabs(qz);
        }
      }
  if (best[0] > best[1]) { const double t = best[0]; best[0] = best[1]; best[1] = t; }
  if (best[1] > best[2]) { const double t = best[1]; best[1] = best[2]; best[2] = t; }
  if (best[0] > best[1]) { const double t = best[0]; best[0] = best[1]; best[1] = t; }
  x[f++] = (float)best[0];
  x[f++] = (float)best[1];
  x[f++] = (float)best[2];
  x[f++] = (float)sqrt(bl);
  x[f++] = (float)log1p(dplus[m]);
  x[f++] = (float)log1p(dminus[m]);
}

// Column mean and population std over the first n_fit rows (FP64, fixed
// order), then every row standardised in place: X <- (X - mu) / sd, with
// sd = 1 where the column is constant on the fit rows.
__global__ __launch_bounds__(256) void standardize_kernel(int n, int n_feat, float* __restrict__ X,
                                                          int n_fit, float* __restrict__ mu_sd) {
  __shared__ double r1[256], r2[256];
  const int col = blockIdx.x, tid = threadIdx.x;
  double s1 = 0.0;
  for (int k = tid; k < n_fit; k += 256) s1 += X[(size_t)k * n_feat + col];
  r1[tid] = s1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) r1[tid] += r1[tid + w];
    __syncthreads();
  }
  const double mean = r1[0] / n_fit;
  double s2 = 0.0;
  for (int k = tid; k < n_fit; k += 256) {
    const double d = X[(size_t)k * n_feat + col] - mean;
    s2 += d * d;
  }
  r2[tid] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) r2[tid] += r2[tid + w];
    __syncthreads();
  }
  const double sd0 = sqrt(r2[0] / n_fit);
  const double sd = sd0 > 1e-10 ? sd0 : 1.0;
  if (tid == 0) {
    mu_sd[2 * col] = (float)mean;
    mu_sd[2 * col + 1] = (float)sd;
  }
  __syncthreads();
  for (int k = tid; k < n; k += 256) {
    float* x = X + (size_t)k * n_feat + col;
    *x = (float)((*x - mean) / sd);
  }
}

// y_k = (ln Gamma[modes[k]] - mu) / sd with mu, sd the mean and population
// std of ln Gamma over the listed modes (FP64).
__global__ __launch_bounds__(256) void targets_kernel(const double* __restrict__ gamma,
                                                      const int32_t* __restrict__ modes, int n,
                                                      float* __restrict__ y, float* __restrict__ mu_sd) {
  __shared__ double r1[256], r2[256];
  const int tid = threadIdx.x;
  double s1 = 0.0;
  for (int k = tid; k < n; k += 256) s1 += log(gamma[modes[k]]);
  r1[tid] = s1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) r1[tid] += r1[tid + w];
    __syncthreads();
  }
  const double mean = r1[0] / n;
  double s2 = 0.0;
  for (int k = tid; k < n; k += 256) {
    const double d = log(gamma[modes[k]]) - mean;
    s2 += d * d;
  }
  r2[tid] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) r2[tid] += r2[tid + w];
    __syncthreads();
  }
  const double sd0 = sqrt(r2[0] / n);
  const double sd = sd0 > 1e-10 ? sd0 : 1.0;
  if (tid == 0) {
    mu_sd[0] = (float)mean;
    mu_sd[1] = (float)sd;
  }
  for (int k = tid; k < n; k += 256) y[k] = (float)((log(gamma[modes[k]]) - mean) / sd);
}

// ----------------------------------------------------------------- MLP
// Flat parameters of one member: W0 [n_in][H], b0 [H], W1..W3 [H][H] each
// followed by its bias, W4 [H] (the head), b4 [1]; row-major.  Hidden
// activations tanh, linear head.
// Offsets are closed forms of the layer index rather than tables: a small
// array indexed by a run-time layer number lives in scratch memory, and every
// lookup in the training loop then becomes a memory load.
struct MlpLayout {
  int n_in, P;
  // layer l < depth maps fan_in -> H (fan_in = n_in for l = 0, else H); the
  // head (l = depth) maps H -> 1
  __host__ __device__ int W(int l) const {
    return l == 0 ? 0 : n_in * kMlpHidden + kMlpHidden + (l - 1) * (kMlpHidden * kMlpHidden + kMlpHidden);
  }
  __host__ __device__ int b(int l) const {
    return W(l) + (l == 0 ? n_in * kMlpHidden : l < kMlpDepth ? kMlpHidden * kMlpHidden : kMlpHidden);
  }
};
__host__ __device__ inline MlpLayout mlp_layout(int n_in) {
  MlpLayout o;
  o.n_in = n_in;
  o.P = o.b(kMlpDepth) + 1;
  return o;
}

// LDS copy of the parameters: weight rows of W0..W3 padded to 65 floats, so
// that W[k][j] is free of bank conflicts both with lanes over j (forward)
// and with lanes over k (backward).
constexpr int kRowPad = kMlpHidden + 1;
struct LdsLayout {
  int n_in, size;
  __host__ __device__ int W(int l) const {
    return l == 0 ? 0 : n_in * kRowPad + kMlpHidden + (l - 1) * (kMlpHidden * kRowPad + kMlpHidden);
  }
  __host__ __device__ int b(int l) const { return W(l) + (l == 0 ? n_in * kRowPad : l < kMlpDepth ? kMlpHidden * kRowPad : kMlpHidden); }
};
__host__ __device__ inline LdsLayout lds_layout(int n_in) {
  LdsLayout o;
  o.n_in = n_in;
  o.size = (o.b(kMlpDepth) + 1 + 3) & ~3;
  return o;
}

// Padded copy of one member's parameters in the training workspace: the
// flat layout above followed by zeros up to a multiple of 64 floats (and at
// least 3 past P), so that every float4 of it is aligned and lies inside one
// weight row or bias of the flat layout.
__host__ __device__ inline int padded_params(int P) { return (P + 3 + 63) / 64 * 64; }
constexpr int kMaxParams = (kMlpMaxIn + 1) * kMlpHidden + (kMlpDepth - 1) * (kMlpHidden + 1) * kMlpHidden +
                           kMlpHidden + 1;
constexpr int kLoadIters = ((kMaxParams + 3) / 4 + kTrainThreads - 1) / kTrainThreads;

// Padded parameters -> LDS layout.  Every load is issued before the first
// LDS store, so the whole vector is in flight at once.
__device__ inline void load_params_lds4(const float* __restrict__ g, float* __restrict__ s,
                                        const MlpLayout& gl, const LdsLayout& sl) {
  const int P = gl.P, n4 = (P + 3) >> 2;
  float4 v[kLoadIters];
#pragma unroll
  for (int i = 0; i < kLoadIters; ++i) {
    const int q = threadIdx.x + i * kTrainThreads;
    v[i] = q < n4 ? reinterpret_cast<const float4*>(g)[q] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int i = 0; i < kLoadIters; ++i) {
    const int f = 4 * (threadIdx.x + i * kTrainThreads);
    if (f < P) {
      int l = 0;
#pragma unroll
      for (int t = 1; t <= kMlpDepth; ++t) l += f >= gl.W(t);
      int dst;
      if (l == kMlpDepth) {
        dst = sl.W(kMlpDepth) + (f - gl.W(kMlpDepth));  // head weights and bias, contiguous
      } else if (f < gl.b(l)) {
        const int r = f - gl.W(l);
        dst = sl.W(l) + (r >> 6) * kRowPad + (r & 63);
      } else {
        dst = sl.b(l) + (f - gl.b(l));
      }
      s[dst] = v[i].x;
      if (f + 1 < P) s[dst + 1] = v[i].y;
      if (f + 2 < P) s[dst + 2] = v[i].z;
      if (f + 3 < P) s[dst + 3] = v[i].w;
    }
  }
}

__device__ __forceinline__ float wave_sum_f(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Barrier of the workgroups of one ensemble member (a cooperative launch
// keeps them all resident).  Every wave first waits for its own memory
// operations (gfx9 counts stores in vmcnt), so that after the workgroup
// barrier one agent-scope release by thread 0 publishes the whole
// workgroup's global writes; thread 0 then arrives on the member's counter
// and polls it.  The wait is bounded: past kSpinCap polls the abort word is
// raised and every workgroup leaves at its next barrier, so the grid always
// drains.  Thread 0's agent-scope acquire invalidates the CU's caches before
// the workgroup reads what others wrote.  The two fences are one-sided
// (release before arriving, acquire after the wait): a full fence at either
// point adds a cache write-back or invalidate and measured 4.6 us more per
// training step.  Returns false once aborted.
__device__ bool member_barrier(unsigned* bar, int* abort_flag, unsigned target, int* lds_ok) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    int ok = 1;
    atomicAdd(bar, 1u);
    for (unsigned it = 0;; ++it) {
      if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if (it >= kSpinCap) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *lds_ok = ok;
  }
  __syncthreads();
  return *lds_ok != 0;
}

struct TrainArgs {
  int n_in, n, G, steps;
  float lr;
  const float* X;       // [n][n_in]
  const float* y;       // [n]
  const float* counts;  // [M][n]
  float* params;        // [M][P] caller's parameters, read at start, written after the last step
  int Pp;               // padded parameter stride of the workspace arrays
  float* wp;            // [M][Pp] padded working copy of the parameters
  float* m1;            // [M][Pp]
  float* m2;            // [M][Pp]
  float* partial;       // [M][G][Pp]
  float* lpart;         // [M][G]
  float* losses;        // [M][steps] or null
  float* grad_out;      // [M][P] or null: reduced gradient of the last step
  unsigned* bar;        // one counter per member, kBarStride apart
  int* abort_flag;
};

constexpr int kBarStride = 32;  // 128 bytes between member counters
constexpr int kMaxGroups = 8;  // partial gradients (float4) in flight per reduction batch

// Workgroup (g, mem) holds sample rows [g S, g S + S) of member mem and owns
// slice g of its padded parameter vector (whole float4s).  Each step: the
// padded parameters into LDS, forward and backward of its rows, partial
// gradient to global, member barrier; then workgroup g reduces the partial
// gradients of its slice over the G workgroups (fixed order, float4 loads
// all in flight) and applies Adam; member barrier.
template <int S>
__global__ __launch_bounds__(kTrainThreads) void mlp_train_kernel(TrainArgs a) {
  constexpr int H = kMlpHidden;
  constexpr int RPW = S / kTrainWaves;  // rows per wave
  static_assert(RPW >= 1 && RPW * kTrainWaves == S, "rows per workgroup");
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  __shared__ int ok_s;
  __shared__ float red_s[kTrainThreads];
  const int g = blockIdx.x, mem = blockIdx.y, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int n_in = a.n_in, n = a.n, G = a.G;
  const MlpLayout gl = mlp_layout(n_in);
  const LdsLayout sl = lds_layout(n_in);
  const int P = gl.P;
  float* prm = lds;                // sl.size
  float* xs = prm + sl.size;       // [S][kMlpMaxIn]
  float* hs = xs + S * kMlpMaxIn;  // [4][S][H] = a_1..a_4
  float* d0 = hs + 4 * S * H;      // [S][H]
  float* d1 = d0 + S * H;          // [S][H]
  float* od = d1 + S * H;          // [S] output deltas
  float* cy = od + S;              // [S][2] counts and targets of the rows
  unsigned* bar = a.bar + mem * kBarStride;
  const unsigned nblk = gridDim.x;
  unsigned bar_target = 0;
  const int row0 = g * S;
  const int Pp = a.Pp;
  float* gpart = a.partial + ((size_t)mem * G + g) * Pp;
  const float* cnt = a.counts + (size_t)mem * n;
  float* wp = a.wp + (size_t)mem * Pp;
  float* m1 = a.m1 + (size_t)mem * Pp;
  float* m2 = a.m2 + (size_t)mem * Pp;

  // constant inputs of this workgroup and the member's count sum
  for (int idx = tid; idx < S * kMlpMaxIn; idx += kTrainThreads) {
    const int i = idx / kMlpMaxIn, k = idx % kMlpMaxIn;
    xs[idx] = (row0 + i < n && k < n_in) ? a.X[(size_t)(row0 + i) * n_in + k] : 0.0f;
  }
  for (int i = tid; i < S; i += kTrainThreads) {
    const bool in = row0 + i < n;
    cy[2 * i] = in ? a.counts[(size_t)mem * n + row0 + i] : 0.f;
    cy[2 * i + 1] = in ? a.y[row0 + i] : 0.f;
  }
  float cs = 0.f;
  for (int i = tid; i < n; i += kTrainThreads) cs += cnt[i];
  red_s[tid] = cs;
  __syncthreads();
  for (int w = kTrainThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red_s[tid] += red_s[tid + w];
    __syncthreads();
  }
  const float inv_csum = 1.0f / red_s[0];
  __syncthreads();
  // this workgroup's slice of float4s: parameters copied in (zero padding),
  // Adam moments zero; a barrier publishes the whole padded vector
  const int n4 = Pp / 4, chunk = (n4 + G - 1) / G;
  const int q_lo = min(n4, g * chunk), q_hi = min(n4, q_lo + chunk);
  const float* gp = a.params + (size_t)mem * P;
  for (int q = q_lo + tid; q < q_hi; q += kTrainThreads) {
    const int p = 4 * q;
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 v = make_float4(p < P ? gp[p] : 0.f, p + 1 < P ? gp[p + 1] : 0.f,
                                 p + 2 < P ? gp[p + 2] : 0.f, p + 3 < P ? gp[p + 3] : 0.f);
    reinterpret_cast<float4*>(wp)[q] = v;
    reinterpret_cast<float4*>(m1)[q] = z;
    reinterpret_cast<float4*>(m2)[q] = z;
  }
  bar_target += nblk;
  if (!member_barrier(bar, a.abort_flag, bar_target, &ok_s)) return;
  float b1t = 1.f, b2t = 1.f;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;

  for (int step = 0; step < a.steps; ++step) {
    load_params_lds4(wp, prm, gl, sl);
    __syncthreads();
    // forward: a_{l+1} = tanh(a_l W_l + b_l); lane = output unit, wave = rows
    for (int l = 0; l < kMlpDepth; ++l) {
      const int K = l == 0 ? n_in : H;
      const float* A = l == 0 ? xs : hs + (l - 1) * S * H;
      const int lda = l == 0 ? kMlpMaxIn : H;
      const float* W = prm + sl.W(l);
      float acc[RPW];
      const float bj = prm[sl.b(l) + lane];
#pragma unroll
      for (int u = 0; u < RPW; ++u) acc[u] = bj;
      int k = 0;
      for (; k + 4 <= K; k += 4) {
        const float w0 = W[k * kRowPad + lane], w1 = W[(k + 1) * kRowPad + lane];
        const float w2 = W[(k + 2) * kRowPad + lane], w3 = W[(k + 3) * kRowPad + lane];
#pragma unroll
        for (int u = 0; u < RPW; ++u) {
          const float4 av = *reinterpret_cast<const float4*>(A + (wv + kTrainWaves * u) * lda + k);
          acc[u] += av.x * w0;
          acc[u] += av.y * w1;
          acc[u] += av.z * w2;
          acc[u] += av.w * w3;
        }
      }
      for (; k < K; ++k) {
        const float w = W[k * kRowPad + lane];
#pragma unroll
        for (int u = 0; u < RPW; ++u) acc[u] += A[(wv + kTrainWaves * u) * lda + k] * w;
      }
      float* Z = hs + l * S * H;
#pragma unroll
      for (int u = 0; u < RPW; ++u) Z[(wv + kTrainWaves * u) * H + lane] = tanhf(acc[u]);
      __syncthreads();
    }
    // head, loss and output delta
    const float* a4 = hs + 3 * S * H;
    const float w4 = prm[sl.W(kMlpDepth) + lane];
    const float b4 = prm[sl.b(kMlpDepth)];
    float lsum = 0.f;
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
      const int i = wv + kTrainWaves * u;
      const float o = wave_sum_f(a4[i * H + lane] * w4) + b4;
      if (lane == 0) {
        const float c = cy[2 * i];
        const float r = row0 + i < n ? o - cy[2 * i + 1] : 0.f;
        od[i] = 2.f * c * r * inv_csum;
        lsum += c * r * r;
      }
    }
    if (lane == 0) red_s[wv] = lsum;
    __syncthreads();
    if (tid == 0) {
      float t = 0.f;
#pragma unroll
      for (int w = 0; w < kTrainWaves; ++w) t += red_s[w];
      a.lpart[(size_t)mem * G + g] = t;
    }
    // head gradient, and delta_3 = od W4 (1 - a4^2)
    if (tid < H) {
      float s = 0.f;
      for (int i = 0; i < S; ++i) s += a4[i * H + tid] * od[i];
      gpart[gl.W(kMlpDepth) + tid] = s;
    } else if (tid == H) {
      float s = 0.f;
      for (int i = 0; i < S; ++i) s += od[i];
      gpart[gl.b(kMlpDepth)] = s;
    }
#pragma unroll
    for (int u = 0; u < RPW; ++u) {
      const int i = wv + kTrainWaves * u;
      const float av = a4[i * H + lane];
      d0[i * H + lane] = od[i] * w4 * (1.f - av * av);
    }
    __syncthreads();
    float* dc = d0;
    float* dn = d1;
    for (int l = kMlpDepth - 1; l >= 0; --l) {
      const int K = l == 0 ? n_in : H;
      const float* A = l == 0 ? xs : hs + (l - 1) * S * H;
      const int lda = l == 0 ? kMlpMaxIn : H;
      // dW_l[k][j] = sum_i a_l[i][k] delta_l[i][j]   (lane = j; waves take
      // blocks of four k; input columns past K are read but never stored)
      for (int k0 = 4 * wv; k0 < K; k0 += 4 * kTrainWaves) {
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
        for (int i = 0; i < S; ++i) {
          const float dv = dc[i * H + lane];
          const float4 av = *reinterpret_cast<const float4*>(A + i * lda + k0);
          s0 += av.x * dv;
          s1 += av.y * dv;
          s2 += av.z * dv;
          s3 += av.w * dv;
        }
        float* gw = gpart + gl.W(l) + k0 * H + lane;
        gw[0] = s0;
        if (k0 + 1 < K) gw[H] = s1;
        if (k0 + 2 < K) gw[2 * H] = s2;
        if (k0 + 3 < K) gw[3 * H] = s3;
      }
      if (tid < H) {
        float s = 0.f;
        for (int i = 0; i < S; ++i) s += dc[i * H + tid];
        gpart[gl.b(l) + tid] = s;
      }
      if (l > 0) {
        // delta_{l-1}[i][k] = (sum_j delta_l[i][j] W_l[k][j]) (1 - a_l[i][k]^2)   (lane = k)
        const float* W = prm + sl.W(l);
        float acc[RPW];
#pragma unroll
        for (int u = 0; u < RPW; ++u) acc[u] = 0.f;
        for (int j = 0; j < H; j += 4) {
          const float w0 = W[lane * kRowPad + j], w1 = W[lane * kRowPad + j + 1];
          const float w2 = W[lane * kRowPad + j + 2], w3 = W[lane * kRowPad + j + 3];
#pragma unroll
          for (int u = 0; u < RPW; ++u) {
            const float4 dv = *reinterpret_cast<const float4*>(dc + (wv + kTrainWaves * u) * H + j);
            acc[u] += dv.x * w0;
            acc[u] += dv.y * w1;
            acc[u] += dv.z * w2;
            acc[u] += dv.w * w3;
          }
        }
#pragma unroll
        for (int u = 0; u < RPW; ++u) {
          const int i = wv + kTrainWaves * u;
          const float av = A[i * H + lane];
          dn[i * H + lane] = acc[u] * (1.f - av * av);
        }
      }
      __syncthreads();
      float* t = dc;
      dc = dn;
      dn = t;
    }
    bar_target += nblk;
    if (!member_barrier(bar, a.abort_flag, bar_target, &ok_s)) return;
    // reduce the partial gradients of this slice in workgroup order and step
    // Adam; all loads of one float4 are issued before the sums.  Padding
    // entries (p >= P) keep a zero gradient and stay zero.
    b1t *= b1;
    b2t *= b2;
    const float c1 = 1.f / (1.f - b1t), c2 = 1.f / (1.f - b2t);
    const bool last = step == a.steps - 1;
    for (int q = q_lo + tid; q < q_hi; q += kTrainThreads) {
      const float4 mo = reinterpret_cast<const float4*>(m1)[q];
      const float4 vo = reinterpret_cast<const float4*>(m2)[q];
      const float4 po = reinterpret_cast<const float4*>(wp)[q];
      float sg[4] = {0.f, 0.f, 0.f, 0.f};
      for (int h0 = 0; h0 < G; h0 += kMaxGroups) {
        float4 v[kMaxGroups];
#pragma unroll
        for (int j = 0; j < kMaxGroups; ++j)
          v[j] = h0 + j < G ? reinterpret_cast<const float4*>(a.partial + ((size_t)mem * G + h0 + j) * Pp)[q]
                            : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int j = 0; j < kMaxGroups; ++j)
          if (h0 + j < G) {
            sg[0] += v[j].x;
            sg[1] += v[j].y;
            sg[2] += v[j].z;
            sg[3] += v[j].w;
          }
      }
      const float mov[4] = {mo.x, mo.y, mo.z, mo.w}, vov[4] = {vo.x, vo.y, vo.z, vo.w};
      const float pov[4] = {po.x, po.y, po.z, po.w};
      float mn[4], vn[4], pn[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int p = 4 * q + e;
        const float sv = p < P ? sg[e] : 0.f;
        mn[e] = b1 * mov[e] + (1.f - b1) * sv;
        vn[e] = b2 * vov[e] + (1.f - b2) * sv * sv;
        pn[e] = pov[e] - a.lr * (mn[e] * c1) / (sqrtf(vn[e] * c2) + eps);
        // the caller's copy only after the last step (the working copy wp
        // carries the parameters between steps)
        if (last && p < P) {
          a.params[(size_t)mem * P + p] = pn[e];
          if (a.grad_out) a.grad_out[(size_t)mem * P + p] = sv;
        }
      }
      reinterpret_cast<float4*>(m1)[q] = make_float4(mn[0], mn[1], mn[2], mn[3]);
      reinterpret_cast<float4*>(m2)[q] = make_float4(vn[0], vn[1], vn[2], vn[3]);
      reinterpret_cast<float4*>(wp)[q] = make_float4(pn[0], pn[1], pn[2], pn[3]);
    }
    if (g == 0 && tid == 0 && a.losses) {
      float s = 0.f;
      for (int h = 0; h < G; ++h) s += a.lpart[(size_t)mem * G + h];
      a.losses[(size_t)mem * a.steps + step] = s * inv_csum;
    }
    bar_target += nblk;
    if (!member_barrier(bar, a.abort_flag, bar_target, &ok_s)) return;
  }
}

__global__ void fill_u32(unsigned* p, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Ensemble forward.  Workgroup = kPredRows rows x M members; wave w runs
// member w over the rows with lanes over hidden units.  Then the mean and
// population std (FP64, member order) of the members' outputs per row.
__global__ __launch_bounds__(64 * kMlpMaxMembers) void mlp_predict_kernel(
    int n_in, int M, int n, const float* __restrict__ X, const float* __restrict__ params,
    float* __restrict__ mean, float* __restrict__ spread) {
  constexpr int H = kMlpHidden, R = kPredRows;
  __shared__ float xs[R * kMlpMaxIn];
  __shared__ float outs[kMlpMaxMembers][R];
  extern __shared__ float hbuf[];  // [M][2][R][H]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row0 = blockIdx.x * R;
  for (int idx = tid; idx < R * n_in; idx += blockDim.x) {
    const int i = idx / n_in, k = idx % n_in;
    xs[i * kMlpMaxIn + k] = row0 + i < n ? X[(size_t)(row0 + i) * n_in + k] : 0.0f;
  }
  __syncthreads();
  const MlpLayout gl = mlp_layout(n_in);
  const float* prm = params + (size_t)wv * gl.P;
  float* h0 = hbuf + (size_t)wv * 2 * R * H;
  float* h1 = h0 + R * H;
  for (int l = 0; l < kMlpDepth; ++l) {
    const int K = l == 0 ? n_in : H;
    const float* A = l == 0 ? xs : h0;
    const int lda = l == 0 ? kMlpMaxIn : H;
    float acc[R];
    const float bj = prm[gl.b(l) + lane];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = bj;
    for (int k = 0; k < K; ++k) {
      const float w = prm[gl.W(l) + k * H + lane];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += A[r * lda + k] * w;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) h1[r * H + lane] = tanhf(acc[r]);
    // the wave alone reads and writes its buffers: a wave-level fence suffices
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float* t = h0;
    h0 = h1;
    h1 = t;
  }
  const float w4 = prm[gl.W(kMlpDepth) + lane];
  const float b4 = prm[gl.b(kMlpDepth)];
  for (int r = 0; r < R; ++r) {
    const float o = wave_sum_f(h0[r * H + lane] * w4) + b4;
    if (lane == 0) outs[wv][r] = o;
  }
  __syncthreads();
  if (tid < R && row0 + tid < n) {
    double s1 = 0.0;
    for (int m = 0; m < M; ++m) s1 += outs[m][tid];
    const double mu = s1 / M;
    double s2 = 0.0;
    for (int m = 0; m < M; ++m) {
      const double d = outs[m][tid] - mu;
      s2 += d * d;
    }
    mean[row0 + tid] = (float)mu;
    spread[row0 + tid] = (float)sqrt(s2 / M);
  }
}

// ----------------------------------------------------------------- gate
// Threshold from held-out rows (one workgroup, FP64).  Row k: weight
// w = star(q) c(omega)/k_B |v|^2, predicted Gamma = exp(mean sd + mu).  Rows
// are taken in ascending gate score (ties as one group); a group is accepted
// while |sum_acc w (1/G_pred - 1/G_true)| <= tol sum_all w / G_true.
// tau = next float above the last accepted score, 0 if none.
__global__ __launch_bounds__(256) void gate_calibrate_kernel(
    int n, const int32_t* __restrict__ modes, const double* __restrict__ gamma,
    const float* __restrict__ mean, const float* __restrict__ y_mu_sd,
    const float* __restrict__ score, const double* __restrict__ omega,
    const double* __restrict__ vel, const int32_t* __restrict__ star, int nb3, double inv_kt_hbar,
    double tol, float* __restrict__ tau_out) {
  __shared__ double diff[kGateMaxRows];
  __shared__ float sp[kGateMaxRows];
  __shared__ int16_t order[kGateMaxRows];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double rs = 0.0;
  for (int k = tid; k < n; k += 256) {
    const int m = modes[k];
    const double x = omega[m] * inv_kt_hbar;
    const double em = expm1(x);
    const double c = x * x * exp(x) / (em * em);
    const double* v = vel + 3 * (size_t)m;
    const double wt = (double)star[m / nb3] * c * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double gt = gamma[m];
    const double gpred = exp((double)mean[k] * (double)y_mu_sd[1] + (double)y_mu_sd[0]);
    diff[k] = wt / gpred - wt / gt;
    sp[k] = score[k];
    rs += wt / gt;
  }
  red[tid] = rs;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double ref = fabs(red[0]);
  for (int k = tid; k < n; k += 256) {
    int pos = 0;
    const float s = sp[k];
    for (int j = 0; j < n; ++j) pos += (sp[j] < s) || (sp[j] == s && j < k);
    order[pos] = (int16_t)k;
  }
  __syncthreads();
  if (tid == 0) {
    double acc = 0.0;
    float tau = 0.0f;
    int r = 0;
    while (r < n) {
      const float s = sp[order[r]];
      double grp = 0.0;
      int e = r;
      while (e < n && sp[order[e]] == s) grp += diff[order[e++]];
      if (!(fabs(acc + grp) <= tol * ref)) break;
      acc += grp;
      tau = nextafterf(s, INFINITY);
      r = e;
    }
    *tau_out = tau;
  }
}

// Domain of the training rows: per column the [min, max] over the first
// n_fit rows; inside[k] = 1 when every feature of row k lies in it.  One
// workgroup.
__global__ __launch_bounds__(256) void domain_kernel(int n, int n_feat, const float* __restrict__ X,
                                                     int n_fit, uint8_t* __restrict__ inside) {
  __shared__ float lo_s[kMlpMaxIn], hi_s[kMlpMaxIn];
  __shared__ float rl[256], rh[256];
  const int tid = threadIdx.x;
  for (int col = 0; col < n_feat; ++col) {
    float lo = INFINITY, hi = -INFINITY;
    for (int k = tid; k < n_fit; k += 256) {
      const float v = X[(size_t)k * n_feat + col];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
    rl[tid] = lo;
    rh[tid] = hi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        rl[tid] = fminf(rl[tid], rl[tid + w]);
        rh[tid] = fmaxf(rh[tid], rh[tid + w]);
      }
      __syncthreads();
    }
    if (tid == 0) {
      lo_s[col] = rl[0];
      hi_s[col] = rh[0];
    }
    __syncthreads();
  }
  for (int k = tid; k < n; k += 256) {
    bool in = true;
    for (int col = 0; col < n_feat; ++col) {
      const float v = X[(size_t)k * n_feat + col];
      in = in && v >= lo_s[col] && v <= hi_s[col];
    }
    inside[k] = in ? 1 : 0;
  }
}

// Gate score of row k: the first-order conductivity error the network's
// disagreement implies, (w / G_pred) spread sd with w = star(q) c/k_B |v|^2
// and G_pred = exp(mean sd + mu); +inf for rows outside the training domain.
__global__ void gate_score_kernel(int n, const int32_t* __restrict__ modes, const float* __restrict__ mean,
                                  const float* __restrict__ spread, const float* __restrict__ y_mu_sd,
                                  const double* __restrict__ omega, const double* __restrict__ vel,
                                  const int32_t* __restrict__ star, int nb3, double inv_kt_hbar,
                                  const uint8_t* __restrict__ inside, float* __restrict__ score) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (inside && !inside[k]) {
    score[k] = INFINITY;
    return;
  }
  const int m = modes[k];
  const double x = omega[m] * inv_kt_hbar;
  const double em = expm1(x);
  const double c = x * x * exp(x) / (em * em);
  const double* v = vel + 3 * (size_t)m;
  const double wt = (double)star[m / nb3] * c * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double sd = y_mu_sd[1];
  const double gpred = exp((double)mean[k] * sd + (double)y_mu_sd[0]);
  score[k] = (float)(wt / gpred * (double)spread[k] * sd);
}

// Rows k with score >= tau whose mode is not yet computed are appended, in
// row order, to `fallback` and marked computed.
__global__ __launch_bounds__(1024) void gate_select_kernel(int n, int n_modes, const int32_t* __restrict__ modes,
                                                           const float* __restrict__ score,
                                                           const float* __restrict__ tau_p,
                                                           uint8_t* __restrict__ computed,
                                                           int32_t* __restrict__ fallback,
                                                           int32_t* __restrict__ n_fallback) {
  __shared__ int wave_tot[16];
  __shared__ int carry;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const float tau = *tau_p;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int k = base + tid;
    const int m = k < n ? modes[k] : 0;
    const bool in_range = m >= 0 && m < n_modes;  // rows of other indices are skipped
    const int f = (k < n && in_range && !(score[k] < tau) && !computed[m]) ? 1 : 0;
    int incl = f;
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wave_tot[wv] = incl;
    __syncthreads();
    int o = carry, tot = 0;
    for (int w = 0; w < 16; ++w) {
      o += (w < wv) ? wave_tot[w] : 0;
      tot += wave_tot[w];
    }
    if (f) {
      fallback[o + incl - 1] = m;
      computed[m] = 1;
    }
    __syncthreads();
    if (tid == 0) carry += tot;
    __syncthreads();
  }
  if (tid == 0) *n_fallback = carry;
}

// Gamma of rows whose mode is not computed: exp(mean sd + mu).
__global__ void fill_kernel(int n, int n_modes, const int32_t* __restrict__ modes, const float* __restrict__ mean,
                            const float* __restrict__ y_mu_sd, const uint8_t* __restrict__ computed,
                            double* __restrict__ gamma) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int m = modes[k];
  if (m < 0 || m >= n_modes) return;  // rows of other indices are skipped
  if (!computed[m]) gamma[m] = exp((double)mean[k] * (double)y_mu_sd[1] + (double)y_mu_sd[0]);
}

// Star map: Gamma(q, s) = mean of Gamma(rep(q), s') over the frequency cluster
// (|d nu| < 1e-4 THz) of s at the representative.
__global__ void star_kernel(int nq, int nb3, const int32_t* __restrict__ ir_of_q,
                            const double* __restrict__ omega, const double* __restrict__ gamma_ir,
                            double* __restrict__ gamma) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nq * nb3) return;
  const int q = m / nb3, s = m % nb3;
  const int r = ir_of_q[q];
  const double* w = omega + (size_t)r * nb3;
  int lo = s, hi = s;
  while (lo > 0 && (w[lo] - w[lo - 1]) / kTwoPi < kDegTolThz) --lo;
  while (hi < nb3 - 1 && (w[hi + 1] - w[hi]) / kTwoPi < kDegTolThz) ++hi;
  double acc = 0.0;
  for (int k = lo; k <= hi; ++k) acc += gamma_ir[(size_t)r * nb3 + k];
  gamma[m] = acc / (hi - lo + 1);
}

template <int S>
size_t train_lds_bytes(int n_in) {
  return sizeof(float) * ((size_t)lds_layout(n_in).size + S * kMlpMaxIn + 6 * S * kMlpHidden + 3 * S);
}

template <int S>
int launch_train(const TrainArgs& a, int M, hipStream_t st, bool* too_large) {
  *too_large = false;
  const size_t lds = train_lds_bytes<S>(a.n_in);
  int dev = 0, n_cu = 0, per_cu = 0, lds_max = 0, coop = 0;
  KALDO_HIP(hipGetDevice(&dev));
  KALDO_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  KALDO_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  KALDO_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop) {
    set_error("kaldo_mlp_train: device has no cooperative launch");
    return KALDO_EUNSUPPORTED;
  }
  if (lds > (size_t)lds_max) {
    *too_large = true;
    return KALDO_OK;
  }
  KALDO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mlp_train_kernel<S>, kTrainThreads, lds));
  if ((long)a.G * M > (long)per_cu * n_cu) {
    *too_large = true;
    return KALDO_OK;
  }
  TrainArgs args = a;
  void* kargs[] = {&args};
  const bool p = prof_on();
  if (p) prof_mark("mlp_train", st, true);
  KALDO_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(mlp_train_kernel<S>),
                                       dim3(a.G, M), dim3(kTrainThreads), kargs, lds, st));
  if (p) prof_mark("mlp_train", st, false);
  return KALDO_OK;
}

}  // namespace kaldo

using namespace kaldo;

// Workspace: phys and sel flags (N_q 3N_b bytes each), the FP32 mode copies,
// the live-q list, its inverse and count, and the per-(q, chunk) sums.
struct JdosWs {
  size_t phys, sel, modef, qlist, part, total;
};
static JdosWs jdos_ws(size_t nq, size_t nm) {
  JdosWs w;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  w.phys = take(nm);
  w.sel = take(nm);
  w.modef = take(sizeof(float4) * nm);
  w.qlist = take(sizeof(int32_t) * (2 * nq + 1));
  w.part = take(sizeof(double) * nq * kFusedMaxChunks * 32);
  w.total = o;
  return w;
}

extern "C" size_t kaldo_jdos_workspace(const kaldo_crystal* c, const int32_t* mesh) {
  if (!c || !mesh || mesh[0] < 1 || mesh[1] < 1 || mesh[2] < 1) return 0;
  const size_t nq = (size_t)mesh[0] * mesh[1] * mesh[2];
  return jdos_ws(nq, nq * c->nb3).total;
}

extern "C" int kaldo_jdos(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                          const double* vel, const kaldo_broadening* b,
                          const int32_t* modes_subset, int64_t n_subset, void* workspace,
                          size_t workspace_bytes, double* dplus, double* dminus, void* stream) {
  KALDO_REQUIRE(c && mesh && omega && vel && b && dplus && dminus, "kaldo_jdos: NULL argument");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "kaldo_jdos: mesh must be >= 1");
  KALDO_REQUIRE(c->nb3 <= kMaxNb3Linewidths, "kaldo_jdos: 3 N_b > 16");
  const int rc = check_broadening(b, true);
  if (rc) return rc;
  KALDO_REQUIRE(n_subset >= 0 && (n_subset == 0 || modes_subset), "kaldo_jdos: bad subset");
  const long nq_l = (long)mesh[0] * mesh[1] * mesh[2];
  KALDO_REQUIRE(nq_l <= 65535L, "kaldo_jdos: mesh too large (N_q > 65535)");
  const size_t need = kaldo_jdos_workspace(c, mesh);
  KALDO_REQUIRE(workspace && workspace_bytes >= need, "kaldo_jdos: workspace too small");
  if (modes_subset && n_subset == 0) return KALDO_OK;
  const int nq = (int)nq_l;
  const int nm = nq * c->nb3;
  const JdosWs w = jdos_ws(nq, nm);
  auto* base = static_cast<unsigned char*>(workspace);
  uint8_t* phys = base + w.phys;
  uint8_t* sel = base + w.sel;
  auto* modef = reinterpret_cast<float4*>(base + w.modef);
  auto* qlist = reinterpret_cast<int32_t*>(base + w.qlist);
  auto* part = reinterpret_cast<double*>(base + w.part);
  int32_t* live_list = qlist;
  int32_t* idx_of_q = qlist + nq;
  int32_t* n_live = qlist + 2 * nq;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KALDO_LAUNCH("jdos_prepare", jdos_prepare, dim3((nm + 255) / 256), dim3(256), 0, st, nm, omega, vel,
               b->nu_min_thz, phys, sel, modef, modes_subset ? 0 : 1, c->d_flags);
  if (modes_subset)
    KALDO_LAUNCH("jdos_select", jdos_select, dim3((unsigned)((n_subset + 255) / 256)), dim3(256), 0,
                 st, modes_subset, (long)n_subset, nm, sel, c->d_flags);
  if (modes_subset)
    KALDO_LAUNCH("lw_live_q", lw_live_q<>, dim3(1), dim3(1024), 0, st, nq, c->nb3, phys, sel,
                 live_list, idx_of_q, n_live);
  else
    KALDO_LAUNCH("lw_all_q", lw_all_q<>, dim3((nq + 255) / 256), dim3(256), 0, st, nq, live_list,
                 idx_of_q, n_live);
  const LwParams p = make_params(c, mesh, 300.0, b);
  // work items (live q, chunk) as in the crystal linewidths: the grid covers
  // min(N_q, n_subset) q-points, the chunk count assumes n_subset / 3N_b
  const long upper = modes_subset ? std::min<long>(nq, n_subset) : nq;
  const long guess = modes_subset ? std::max<long>(1, n_subset / c->nb3) : nq;
  const int max_chunks =
      (int)std::max<long>(1, std::min<long>(kFusedMaxChunks, (long)nq * c->nb3 / (2 * kJdosThreads)));
  const int n_chunk =
      std::min(fused_chunks((int)std::min<long>(guess, 1l << 30), kWorkItems), max_chunks);
  const dim3 grid((unsigned)(upper * n_chunk));
  if (c->nb3 <= 8)
    KALDO_LAUNCH("jdos_kernel", jdos_kernel<8>, grid, dim3(kJdosThreads), 0, st, p, omega, vel, modef,
                 phys, sel, live_list, n_live, n_chunk, part);
  else
    KALDO_LAUNCH("jdos_kernel", jdos_kernel<16>, grid, dim3(kJdosThreads), 0, st, p, omega, vel, modef,
                 phys, sel, live_list, n_live, n_chunk, part);
  KALDO_LAUNCH("jdos_finish", jdos_finish, dim3((nm + 255) / 256), dim3(256), 0, st, nm, c->nb3, nq,
               phys, sel, idx_of_q, n_chunk, part, dplus, dminus);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int32_t kaldo_surrogate_feature_count(const kaldo_crystal* c) {
  return c ? c->nb3 + 8 : -1;
}

extern "C" int kaldo_surrogate_features(const kaldo_crystal* c, const int32_t* mesh,
                                        const double* omega, const double* vel,
                                        const double* dplus, const double* dminus,
                                        const int32_t* modes, int64_t n, float* features,
                                        void* stream) {
  KALDO_REQUIRE(c && mesh && omega && vel && dplus && dminus, "kaldo_surrogate_features: NULL argument");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "kaldo_surrogate_features: mesh must be >= 1");
  KALDO_REQUIRE(n >= 0 && n < (1l << 31) && (n == 0 || (modes && features)),
                "kaldo_surrogate_features: bad rows");
  KALDO_REQUIRE(c->nb3 + 8 <= kMlpMaxIn, "kaldo_surrogate_features: 3 N_b + 8 > 32");
  if (n == 0) return KALDO_OK;
  double rc[9];
  reciprocal(c->lattice, rc);
  const double3 b0 = make_double3(rc[0], rc[1], rc[2]), b1 = make_double3(rc[3], rc[4], rc[5]),
                b2 = make_double3(rc[6], rc[7], rc[8]);
  KALDO_LAUNCH("features_kernel", features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
               static_cast<hipStream_t>(stream), c->nb3, mesh[0], mesh[1], mesh[2], b0, b1, b2,
               omega, vel, dplus, dminus, modes, (int)n, c->nb3 + 8, features);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_standardize(int64_t n, int32_t n_feat, float* X, int64_t n_fit, float* mu_sd,
                                 void* stream) {
  KALDO_REQUIRE(X && mu_sd && n_feat > 0 && n_fit > 0 && n_fit <= n && n < (1l << 31),
                "kaldo_standardize: bad arguments");
  KALDO_LAUNCH("standardize_kernel", standardize_kernel, dim3(n_feat), dim3(256), 0,
               static_cast<hipStream_t>(stream), (int)n, n_feat, X, (int)n_fit, mu_sd);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_surrogate_targets(const double* gamma, const int32_t* modes, int64_t n,
                                       float* y, float* y_mu_sd, void* stream) {
  KALDO_REQUIRE(gamma && modes && y && y_mu_sd && n > 0 && n < (1l << 31),
                "kaldo_surrogate_targets: bad arguments");
  KALDO_LAUNCH("targets_kernel", targets_kernel, dim3(1), dim3(256), 0,
               static_cast<hipStream_t>(stream), gamma, modes, (int)n, y, y_mu_sd);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int32_t kaldo_mlp_param_count(int32_t n_in) {
  return n_in > 0 && n_in <= kMlpMaxIn ? mlp_layout(n_in).P : -1;
}

static size_t train_groups(int32_t n, int S) { return ((size_t)n + S - 1) / S; }

// Workspace head: one barrier counter per member (kBarStride words apart),
// then the abort word; 256-byte aligned.
static size_t train_head_bytes(int32_t n_members) {
  return ((size_t)(n_members + 1) * kBarStride * 4 + 255) / 256 * 256;
}

extern "C" size_t kaldo_mlp_workspace(int32_t n_in, int32_t n_members, int32_t n_samples) {
  if (n_in <= 0 || n_in > kMlpMaxIn || n_members <= 0 || n_samples <= 0) return 0;
  const size_t Pp = padded_params(mlp_layout(n_in).P);
  const size_t G = train_groups(n_samples, 8);  // the largest grid the launcher may choose
  const size_t floats = 3 * Pp * n_members + G * Pp * n_members + G * n_members;
  return train_head_bytes(n_members) + (floats * sizeof(float) + 255) / 256 * 256;
}

extern "C" int kaldo_mlp_train(int32_t n_in, int32_t n_members, int32_t n_samples, const float* X,
                               const float* y, const float* counts, float* params, int32_t steps,
                               float lr, void* workspace, size_t workspace_bytes, float* losses,
                               float* grad_out, void* stream) {
  KALDO_REQUIRE(n_in > 0 && n_in <= kMlpMaxIn, "kaldo_mlp_train: n_in must be in [1, 32]");
  KALDO_REQUIRE(n_members > 0 && n_samples > 0 && steps >= 0, "kaldo_mlp_train: bad sizes");
  KALDO_REQUIRE(X && y && counts && params && workspace, "kaldo_mlp_train: NULL argument");
  KALDO_REQUIRE(std::isfinite(lr) && lr > 0, "kaldo_mlp_train: lr must be > 0");
  KALDO_REQUIRE(workspace_bytes >= kaldo_mlp_workspace(n_in, n_members, n_samples),
                "kaldo_mlp_train: workspace too small");
  if (steps == 0) return KALDO_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t P = mlp_layout(n_in).P;
  auto* base = static_cast<char*>(workspace);
  const size_t head = train_head_bytes(n_members);
  auto* bar = reinterpret_cast<unsigned*>(base);
  auto* abort_flag = reinterpret_cast<int*>(base + (size_t)n_members * kBarStride * 4);
  float* f = reinterpret_cast<float*>(base + head);
  const int head_words = (int)(head / 4);
  KALDO_LAUNCH("fill_u32", fill_u32, dim3((head_words + 255) / 256), dim3(256), 0, st, bar, head_words, 0u);
  TrainArgs a;
  a.n_in = n_in;
  a.n = n_samples;
  a.steps = steps;
  a.lr = lr;
  a.X = X;
  a.y = y;
  a.counts = counts;
  a.params = params;
  const size_t Pp = padded_params((int)P);
  a.Pp = (int)Pp;
  a.wp = f;
  a.m1 = f + Pp * n_members;
  a.m2 = f + 2 * Pp * n_members;
  a.losses = losses;
  a.grad_out = grad_out;
  a.bar = bar;
  a.abort_flag = abort_flag;
  bool too_large = true;
  int rc = KALDO_OK;
  // fewest rows per workgroup whose grid fits on the device at once
  for (int S : {8, 16, 32}) {
    a.G = (int)train_groups(n_samples, S);
    a.partial = f + 3 * Pp * n_members;
    a.lpart = a.partial + (size_t)a.G * Pp * n_members;
    if (S == 8) rc = launch_train<8>(a, n_members, st, &too_large);
    if (S == 16) rc = launch_train<16>(a, n_members, st, &too_large);
    if (S == 32) rc = launch_train<32>(a, n_members, st, &too_large);
    if (rc != KALDO_OK || !too_large) break;
  }
  if (rc != KALDO_OK) return rc;
  if (too_large) {
    set_error("kaldo_mlp_train: members x sample groups exceed the co-resident workgroups");
    return KALDO_EUNSUPPORTED;
  }
  KALDO_HIP(hipGetLastError());
  int aborted = 0;
  KALDO_HIP(hipMemcpyAsync(&aborted, abort_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  KALDO_HIP(hipStreamSynchronize(st));
  if (aborted) {
    set_error("kaldo_mlp_train: grid barrier timed out");
    return KALDO_EDEVICE;
  }
  return KALDO_OK;
}

extern "C" int kaldo_mlp_predict(int32_t n_in, int32_t n_members, int64_t n, const float* X,
                                 const float* params, float* mean, float* spread, void* stream) {
  KALDO_REQUIRE(n_in > 0 && n_in <= kMlpMaxIn, "kaldo_mlp_predict: n_in must be in [1, 32]");
  KALDO_REQUIRE(n_members > 0 && n_members <= kMlpMaxMembers, "kaldo_mlp_predict: members in [1, 16]");
  KALDO_REQUIRE(n >= 0 && n < (1l << 31), "kaldo_mlp_predict: bad row count");
  KALDO_REQUIRE(n == 0 || (X && params && mean && spread), "kaldo_mlp_predict: NULL argument");
  if (n == 0) return KALDO_OK;
  KALDO_LAUNCH("mlp_predict", mlp_predict_kernel, dim3((unsigned)((n + kPredRows - 1) / kPredRows)),
               dim3(64 * n_members), sizeof(float) * 2 * kPredRows * kMlpHidden * n_members,
               static_cast<hipStream_t>(stream), n_in, n_members, (int)n, X,
               params, mean, spread);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_gate_calibrate(int64_t n, const int32_t* modes, const double* gamma,
                                    const float* mean, const float* y_mu_sd, const float* score,
                                    const double* omega, const double* vel, const int32_t* star_size,
                                    int32_t nb3, double temperature, double tol, float* tau,
                                    void* stream) {
  KALDO_REQUIRE(n > 0 && n <= kGateMaxRows, "kaldo_gate_calibrate: rows must be in [1, 4096]");
  KALDO_REQUIRE(modes && gamma && mean && y_mu_sd && score && omega && vel && star_size && tau,
                "kaldo_gate_calibrate: NULL argument");
  KALDO_REQUIRE(nb3 > 0, "kaldo_gate_calibrate: nb3 must be > 0");
  KALDO_REQUIRE(std::isfinite(temperature) && temperature > 0, "kaldo_gate_calibrate: temperature <= 0");
  KALDO_REQUIRE(std::isfinite(tol) && tol >= 0, "kaldo_gate_calibrate: tol < 0");
  KALDO_LAUNCH("gate_calibrate", gate_calibrate_kernel, dim3(1), dim3(256), 0,
               static_cast<hipStream_t>(stream), (int)n, modes, gamma, mean, y_mu_sd, score, omega,
               vel, star_size, nb3, kHbar / (kKb * temperature), tol, tau);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_surrogate_domain(int64_t n, int32_t n_feat, const float* X, int64_t n_fit,
                                      uint8_t* inside, void* stream) {
  KALDO_REQUIRE(X && inside && n_feat > 0 && n_feat <= kMlpMaxIn && n_fit > 0 && n_fit <= n &&
                    n < (1l << 31),
                "kaldo_surrogate_domain: bad arguments");
  KALDO_LAUNCH("surrogate_domain", domain_kernel, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream),
               (int)n, n_feat, X, (int)n_fit, inside);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_gate_score(int64_t n, const int32_t* modes, const float* mean, const float* spread,
                                const float* y_mu_sd, const double* omega, const double* vel,
                                const int32_t* star_size, int32_t nb3, double temperature,
                                const uint8_t* inside, float* score, void* stream) {
  KALDO_REQUIRE(n >= 0 && n < (1l << 31), "kaldo_gate_score: bad row count");
  KALDO_REQUIRE(n == 0 || (modes && mean && spread && y_mu_sd && omega && vel && star_size && score),
                "kaldo_gate_score: NULL argument");
  KALDO_REQUIRE(nb3 > 0, "kaldo_gate_score: nb3 must be > 0");
  KALDO_REQUIRE(std::isfinite(temperature) && temperature > 0, "kaldo_gate_score: temperature <= 0");
  if (n == 0) return KALDO_OK;
  KALDO_LAUNCH("gate_score", gate_score_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
               static_cast<hipStream_t>(stream), (int)n, modes, mean, spread, y_mu_sd, omega, vel,
               star_size, nb3, kHbar / (kKb * temperature), inside, score);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_gate_select(int64_t n, int64_t n_modes, const int32_t* modes, const float* score,
                                 const float* tau, uint8_t* computed, int32_t* fallback,
                                 int32_t* n_fallback, void* stream) {
  KALDO_REQUIRE(n >= 0 && n < (1l << 31) && modes && score && tau && computed && fallback && n_fallback,
                "kaldo_gate_select: bad arguments");
  KALDO_REQUIRE(n_modes >= 1 && n_modes < (1l << 31), "kaldo_gate_select: n_modes out of range");
  KALDO_LAUNCH("gate_select", gate_select_kernel, dim3(1), dim3(1024), 0,
               static_cast<hipStream_t>(stream), (int)n, (int)n_modes, modes, score, tau, computed,
               fallback, n_fallback);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_surrogate_fill(int64_t n, int64_t n_modes, const int32_t* modes,
                                    const float* mean, const float* y_mu_sd,
                                    const uint8_t* computed, double* gamma, void* stream) {
  KALDO_REQUIRE(n >= 0 && n < (1l << 31) && (n == 0 || (modes && mean && y_mu_sd && computed && gamma)),
                "kaldo_surrogate_fill: bad arguments");
  KALDO_REQUIRE(n_modes >= 1 && n_modes < (1l << 31), "kaldo_surrogate_fill: n_modes out of range");
  if (n == 0) return KALDO_OK;
  KALDO_LAUNCH("surrogate_fill", fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
               static_cast<hipStream_t>(stream), (int)n, (int)n_modes, modes, mean, y_mu_sd,
               computed, gamma);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_star_map(const int32_t* mesh, int32_t nb3, const int32_t* ir_of_q,
                              const double* omega, const double* gamma_ir, double* gamma,
                              void* stream) {
  KALDO_REQUIRE(mesh && ir_of_q && omega && gamma_ir && gamma && nb3 > 0, "kaldo_star_map: bad arguments");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "kaldo_star_map: mesh must be >= 1");
  KALDO_REQUIRE(gamma != gamma_ir, "kaldo_star_map: gamma must not alias gamma_ir");
  const int nq = mesh[0] * mesh[1] * mesh[2];
  const int nm = nq * nb3;
  KALDO_LAUNCH("star_map", star_kernel, dim3((nm + 255) / 256), dim3(256), 0,
               static_cast<hipStream_t>(stream), nq, nb3, ir_of_q, omega, gamma_ir, gamma);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

// ----------------------------------------------------------------- host
// Point operations of the crystal: integer matrices M (entries -1, 0, 1 in
// the lattice basis, x -> M x on column fractional coordinates) that keep
// the metric G = A A^T (M^T G M = G) and map the basis onto itself, masses
// included, up to a translation.  On the reciprocal side k -> M^T k (over a
// group the set {M^T} equals {M^-T}); q and M^T q are in one star when M^T q
// lies on the mesh.  ir_of_q[q] = the smallest flat index in the star of q;
// star_size[q] = the star's size at a representative, 0 elsewhere.  Entries
// in -1..1 cover every point operation of a reduced basis.
extern "C" int kaldo_mesh_ibz(const double* lattice, int32_t n_basis, const double* frac,
                              const double* mass, const int32_t* mesh, int32_t* ir_of_q,
                              int32_t* star_size, int32_t* n_ops_out, int32_t* n_ir_out) {
  KALDO_REQUIRE(lattice && frac && mass && mesh && ir_of_q && star_size, "kaldo_mesh_ibz: NULL argument");
  KALDO_REQUIRE(n_basis >= 1, "kaldo_mesh_ibz: n_basis must be >= 1");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "kaldo_mesh_ibz: mesh must be >= 1");
  double G[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      G[3 * i + j] = 0;
      for (int k = 0; k < 3; ++k) G[3 * i + j] += lattice[3 * i + k] * lattice[3 * j + k];
    }
  double gscale = 0;
  for (double v : G) gscale = std::max(gscale, std::fabs(v));
  KALDO_REQUIRE(gscale > 0 && std::isfinite(gscale), "kaldo_mesh_ibz: bad lattice");
  auto wrap = [](double x) { return x - std::nearbyint(x); };
  std::vector<std::array<int, 9>> ops;
  std::array<int, 9> M;  // M[3 r + c]: row r, column c
  for (int code = 0; code < 19683; ++code) {
    int t = code;
    for (int k = 0; k < 9; ++k) {
      M[k] = t % 3 - 1;
      t /= 3;
    }
    bool ok = true;
    for (int i = 0; i < 3 && ok; ++i)
      for (int j = 0; j < 3 && ok; ++j) {
        double s = 0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) s += M[3 * a + i] * G[3 * a + b] * M[3 * b + j];
        ok = std::fabs(s - G[3 * i + j]) <= 1e-9 * gscale;
      }
    if (!ok) continue;
    // the basis must map onto itself: x_a -> M x_a + t for one translation t
    auto image = [&](int a, double* out) {
      for (int r = 0; r < 3; ++r) {
        out[r] = 0;
        for (int c = 0; c < 3; ++c) out[r] += M[3 * r + c] * frac[3 * a + c];
      }
    };
    bool found = false;
    double x0[3];
    image(0, x0);
    for (int j = 0; j < n_basis && !found; ++j) {
      if (std::fabs(mass[j] - mass[0]) > 1e-9 * std::fabs(mass[0])) continue;
      const double tr[3] = {frac[3 * j] - x0[0], frac[3 * j + 1] - x0[1], frac[3 * j + 2] - x0[2]};
      bool all = true;
      for (int a = 0; a < n_basis && all; ++a) {
        double xa[3];
        image(a, xa);
        int hits = 0;
        for (int b = 0; b < n_basis; ++b) {
          if (std::fabs(mass[b] - mass[a]) > 1e-9 * std::fabs(mass[a])) continue;
          if (std::fabs(wrap(frac[3 * b] - xa[0] - tr[0])) < 1e-6 &&
              std::fabs(wrap(frac[3 * b + 1] - xa[1] - tr[1])) < 1e-6 &&
              std::fabs(wrap(frac[3 * b + 2] - xa[2] - tr[2])) < 1e-6)
            ++hits;
        }
        all = hits == 1;
      }
      found = all;
    }
    if (found) ops.push_back(M);
  }
  const int N0 = mesh[0], N1 = mesh[1], N2 = mesh[2];
  const int nq = N0 * N1 * N2;
  // k'_i = sum_j M_ji n_j / N_j; with L = lcm(N): n'_i = t_i N_i / L,
  // t_i = sum_j M_ji n_j (L / N_j), on the mesh when L divides t_i N_i
  auto gcd = [](long a, long b) {
    while (b) {
      const long t = a % b;
      a = b;
      b = t;
    }
    return a;
  };
  long L = N0;
  L = L / gcd(L, N1) * N1;
  L = L / gcd(L, N2) * N2;
  for (int q = 0; q < nq; ++q) {
    const long n[3] = {q / (N1 * N2), (q / N2) % N1, q % N2};
    int best = q;
    for (const auto& R : ops) {
      long m[3];
      bool on = true;
      for (int i = 0; i < 3 && on; ++i) {
        long t = 0;
        for (int j = 0; j < 3; ++j) t += R[3 * j + i] * n[j] * (L / mesh[j]);
        const long num = t * mesh[i];
        on = num % L == 0;
        const long v = num / L;
        m[i] = ((v % mesh[i]) + mesh[i]) % mesh[i];
      }
      if (on) best = std::min(best, (int)((m[0] * N1 + m[1]) * N2 + m[2]));
    }
    ir_of_q[q] = best;
  }
  int n_ir = 0;
  for (int q = 0; q < nq; ++q) star_size[q] = 0;
  for (int q = 0; q < nq; ++q) ++star_size[ir_of_q[q]];
  for (int q = 0; q < nq; ++q) n_ir += ir_of_q[q] == q;
  if (n_ops_out) *n_ops_out = (int32_t)ops.size();
  if (n_ir_out) *n_ir_out = n_ir;
  return KALDO_OK;
}
