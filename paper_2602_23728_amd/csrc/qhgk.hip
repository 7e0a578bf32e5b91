// Quasi-harmonic Green-Kubo conductivity: Eq. qhgk (a Gamma-point solid) and
// the interband term of Eq. qhgk_crystal (a crystal on a mesh),
//   kappa_ab = 1/V sum_{mu nu} c_{mu nu} v^a_{mu nu} tau_{mu nu} v^b_{nu mu},
// with
//   c_{mu nu}   = (hbar/T) w_mu w_nu (n_mu - n_nu)/(w_nu - w_mu), the modal
//                 heat capacity of Eq. heatcap (its limit) for pairs closer
//                 than 1e-4 THz (their mean);
//   v^a_{mu nu} = eta_mu^H (dD/dq_a) eta_nu / (2 sqrt(w_mu w_nu)), dD/dq_a
//                 written with the full separation of the two atoms (lattice
//                 vector plus basis offset; minimum image for one cell);
//   tau_{mu nu} = g/(2((w_mu - w_nu)^2 + g^2)), g = (Gamma_mu + Gamma_nu)/2,
// over modes with nu >= nu_min and Gamma above 1e-8 of the largest.
//
// Crystal (qh_crystal, one workgroup per q): replica phases, the three
// velocity operators in LDS, v = eta^H (dD/dq) eta by two small complex
// products, the weighted pair sums over s != s' and a fixed-order reduction;
// qh_finish adds the q-points in order.
// Gamma point: the operator S_a = D o (R_j - R_i)_a is sparse (bonded
// pairs), so W_a = S_a E is a sparse-times-dense product (qh_csr_*,
// qh_spmm); E^T W_a is the dense part (qh_gemm: FP64 matrix cores, the three
// components of one 64 x 64 tile of mode pairs in one workgroup), whose
// epilogue forms the weighted products and the tile's share of every mode's
// diffusivity, so the velocity matrices are never written out.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace kaldo {

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double qd4;

// c_{mu nu} / k_B; hk = hbar/(k_B T) in ps.
__device__ __forceinline__ double qh_pair_c(double w1, double w2, double n1, double n2, double c1,
                                            double c2, double hk) {
  if (fabs(w2 - w1) / kTwoPi < kDegTolThz) return 0.5 * (c1 + c2);
  return hk * w1 * w2 * (n1 - n2) / (w2 - w1);
}

__device__ __forceinline__ double qh_pair_tau(double w1, double w2, double g1, double g2) {
  const double g = 0.5 * (g1 + g2);
  const double dw = w1 - w2;
  return g / (2.0 * (dw * dw + g * g));
}

// Per mode: active flag (nu >= nu_min, Gamma > floor), population n, heat
// capacity c/k_B and 1/sqrt(2 w); one workgroup also finds max Gamma first.
// Inputs are checked (non-finite -> status; imaginary above nu_min -> status).
__global__ __launch_bounds__(1024) void qh_modes(long n_modes, const double* __restrict__ omega,
                                                 const double* __restrict__ gamma, double hk,
                                                 double nu_min, double4* __restrict__ mode,
                                                 int32_t* __restrict__ flags) {
  __shared__ double red[1024];
  const int t = threadIdx.x;
  double gmax = 0.0, chk = 0.0;
  bool imag = false;
  for (long m = t; m < n_modes; m += 1024) {
    const double g = gamma[m], w = omega[m];
    gmax = fmax(gmax, g);
    chk += (g - g) + (w - w);
    imag = imag || (w < 0.0 && (-w / kTwoPi) >= nu_min);
  }
  if (!(chk == 0.0)) raise_flag(flags, kFlagNonFinite);
  if (imag) raise_flag(flags, kFlagImaginary);
  red[t] = gmax;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  const double floor_g = kGammaFloorRel * red[0];
  for (long m = t; m < n_modes; m += 1024) {
    const double w = omega[m], g = gamma[m];
    const bool act = (w / kTwoPi >= nu_min) && (g > floor_g) && (g > 0.0);
    double n = 0.0, c = 0.0, nrm = 0.0;
    if (act) {
      const double x = w * hk;
      const double em = expm1(x);
      n = 1.0 / em;
      c = x * x * (em + 1.0) / (em * em);
      nrm = 1.0 / sqrt(2.0 * w);
    }
    // (population, heat capacity, 1/sqrt(2 w), active): the product of two
    // modes' third entries is the 1/(2 sqrt(w_mu w_nu)) of their velocity
    mode[m] = make_double4(n, c, nrm, act ? 1.0 : 0.0);
  }
}

// ---------------------------------------------------------------- crystal

struct QhCrystal {
  int nq, nb3, n_rep, N[3];
  double hk, tau_cart[5][3];  // Cartesian basis positions
};

template <int NB3>
__global__ __launch_bounds__(256) void qh_crystal(QhCrystal p, const double* __restrict__ fc2,
                                                  const double* __restrict__ repcart,
                                                  const int32_t* __restrict__ rep,
                                                  const double* __restrict__ omega,
                                                  const double* __restrict__ gamma,
                                                  const double* __restrict__ evec,
                                                  const double4* __restrict__ mode,
                                                  double* __restrict__ part) {
  extern __shared__ double2 ph[];  // e^{-i q.R_l}, [n_rep]
  __shared__ double2 dD[3][NB3][NB3];
  __shared__ double2 eta[NB3][NB3];
  __shared__ double2 T[3][NB3][NB3];
  __shared__ double red[256][6];
  const int q = blockIdx.x, tid = threadIdx.x;
  const int N0 = p.N[0], N1 = p.N[1], N2 = p.N[2];
  const int a0 = q / (N1 * N2), a1 = (q / N2) % N1, a2 = q % N2;
  for (int l = tid; l < p.n_rep; l += 256) {
    const int32_t* r = rep + 3 * l;
    const int m0 = ((a0 * r[0]) % N0 + N0) % N0, m1 = ((a1 * r[1]) % N1 + N1) % N1,
              m2 = ((a2 * r[2]) % N2 + N2) % N2;
    const double f = (double)m0 / N0 + (double)m1 / N1 + (double)m2 / N2;
    double sn, cs;
    sincospi(-2.0 * f, &sn, &cs);
    ph[l] = make_double2(cs, sn);
  }
  for (int k = tid; k < NB3 * NB3; k += 256) {
    const int r = k / NB3, s = k % NB3;
    const size_t o = (((size_t)q * NB3 + r) * NB3 + s) * 2;
    eta[r][s] = make_double2(evec[o], evec[o + 1]);
  }
  __syncthreads();
  // dD/dq_a [r][c] = sum_l -i sep_a e^{-i q.R_l} D(0 i, l j), in ps^-2 A
  for (int k = tid; k < NB3 * NB3; k += 256) {
    const int r = k / NB3, c = k % NB3;
    const int i = r / 3, j = c / 3;
    double re[3] = {0, 0, 0}, im[3] = {0, 0, 0};
    for (int l = 0; l < p.n_rep; ++l) {
      const double f = fc2[((size_t)r * p.n_rep + l) * NB3 + c] * kU;
      if (f == 0.0) continue;
      const double2 e = ph[l];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double sep = repcart[3 * l + a] + p.tau_cart[j][a] - p.tau_cart[i][a];
        // -i sep f (e.x + i e.y) = sep f e.y - i sep f e.x
        re[a] += sep * f * e.y;
        im[a] -= sep * f * e.x;
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) dD[a][r][c] = make_double2(re[a], im[a]);
  }
  __syncthreads();
  // T_a = dD_a eta
  for (int k = tid; k < 3 * NB3 * NB3; k += 256) {
    const int a = k / (NB3 * NB3), r = (k / NB3) % NB3, n = k % NB3;
    double tr = 0.0, ti = 0.0;
#pragma unroll
    for (int c = 0; c < NB3; ++c) {
      const double2 x = dD[a][r][c], y = eta[c][n];
      tr += x.x * y.x - x.y * y.y;
      ti += x.x * y.y + x.y * y.x;
    }
    T[a][r][n] = make_double2(tr, ti);
  }
  __syncthreads();
  // V_a[m][n] = eta^H T_a, normalised; weighted pair products over m != n
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int k = tid; k < NB3 * NB3; k += 256) {
    const int m = k / NB3, n = k % NB3;
    if (m == n) continue;
    const double4 dm = mode[(size_t)q * NB3 + m], dn = mode[(size_t)q * NB3 + n];
    if (dm.w == 0.0 || dn.w == 0.0) continue;
    double vr[3], vi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int r = 0; r < NB3; ++r) {
        const double2 x = eta[r][m], y = T[a][r][n];
        // conj(x) y
        sr += x.x * y.x + x.y * y.y;
        si += x.x * y.y - x.y * y.x;
      }
      vr[a] = sr * dm.z * dn.z;
      vi[a] = si * dm.z * dn.z;
    }
    const double w1 = omega[(size_t)q * NB3 + m], w2 = omega[(size_t)q * NB3 + n];
    const double wt = qh_pair_c(w1, w2, dm.x, dn.x, dm.y, dn.y, p.hk) *
                      qh_pair_tau(w1, w2, gamma[(size_t)q * NB3 + m], gamma[(size_t)q * NB3 + n]);
    // Re(v_a conj(v_b))
    acc[0] += wt * (vr[0] * vr[0] + vi[0] * vi[0]);
    acc[1] += wt * (vr[0] * vr[1] + vi[0] * vi[1]);
    acc[2] += wt * (vr[0] * vr[2] + vi[0] * vi[2]);
    acc[3] += wt * (vr[1] * vr[1] + vi[1] * vi[1]);
    acc[4] += wt * (vr[1] * vr[2] + vi[1] * vi[2]);
    acc[5] += wt * (vr[2] * vr[2] + vi[2] * vi[2]);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) red[tid][k] = acc[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int k = 0; k < 6; ++k) red[tid][k] += red[tid + w][k];
    __syncthreads();
  }
  if (tid < 6) part[(size_t)q * 6 + tid] = red[0][tid];
}

// kappa[9] = scale * sum of the n_part partial 6-vectors: thread t sums the
// partials t, t + 256, ... in order, then a fixed tree over the threads.
__global__ __launch_bounds__(256) void qh_finish(long n_part, const double* __restrict__ part,
                                                 double scale, double* __restrict__ kappa) {
  __shared__ double red[256][6];
  __shared__ double out[6];
  const int t = threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long i = t; i < n_part; i += 256)
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += part[i * 6 + k];
#pragma unroll
  for (int k = 0; k < 6; ++k) red[t][k] = acc[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int k = 0; k < 6; ++k) red[t][k] += red[t + w][k];
    __syncthreads();
  }
  if (t < 6) out[t] = scale * red[0][t];
  __syncthreads();
  if (t == 0) {
    const int map[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
    for (int i = 0; i < 9; ++i) kappa[i] = out[map[i]];
  }
}

// ---------------------------------------------------------------- Gamma point

// Nonzero count of row r of D (3N x 3N, dense) over columns of other atoms.
__global__ void qh_csr_count(int n3, const double* __restrict__ D, int32_t* __restrict__ cnt) {
  const int r = blockIdx.x, lane = threadIdx.x;
  int c_own = 0;
  for (int c = lane; c < n3; c += 64) c_own += (D[(size_t)r * n3 + c] != 0.0 && c / 3 != r / 3);
  for (int off = 32; off > 0; off >>= 1) c_own += __shfl_xor(c_own, off, 64);
  if (lane == 0) cnt[r] = c_own;
}

// Exclusive scan of the row counts (one workgroup, sequential runs per thread).
__global__ __launch_bounds__(1024) void qh_csr_scan(int n, const int32_t* __restrict__ cnt,
                                                    int32_t* __restrict__ ptr) {
  __shared__ int sums[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  int own = 0;
  for (int i = lo; i < hi; ++i) own += cnt[i];
  sums[t] = own;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? sums[t - off] : 0;
    __syncthreads();
    sums[t] += v;
    __syncthreads();
  }
  int run = sums[t] - own;
  for (int i = lo; i < hi; ++i) {
    ptr[i] = run;
    run += cnt[i];
  }
  if (t == 1023) ptr[n] = sums[1023];
}

// Row r of S_a = D o sep_a (ps^-2 A), columns ascending: one wave per row,
// 64 columns per round compacted by a wave-wide prefix of the nonzero flags.
__global__ void qh_csr_fill(int n3, const double* __restrict__ D, const double* __restrict__ frac,
                            const double* __restrict__ lat, const int32_t* __restrict__ ptr,
                            int32_t* __restrict__ col, double4* __restrict__ val) {
  const int r = blockIdx.x, lane = threadIdx.x;
  const int i = r / 3;
  int base = ptr[r];
  for (int c0 = 0; c0 < n3; c0 += 64) {
    const int c = c0 + lane;
    const double d = c < n3 ? D[(size_t)r * n3 + c] : 0.0;
    const bool nz = c < n3 && d != 0.0 && c / 3 != i;
    const unsigned long long mask = __ballot(nz);
    if (nz) {
      const int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
      const int j = c / 3;
      double f[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double x = frac[3 * j + k] - frac[3 * i + k];
        f[k] = x - rint(x);  // minimum image
      }
      double s[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) s[a] = f[0] * lat[a] + f[1] * lat[3 + a] + f[2] * lat[6 + a];
      const double dk = d * kU;
      col[pos] = c;
      val[pos] = make_double4(dk * s[0], dk * s[1], dk * s[2], 0.0);
    }
    base += __popcll(mask);
  }
}

// W_a[r][nu] = sum_c S_a[r][c] E[c][nu], one workgroup per row r.
__global__ __launch_bounds__(256) void qh_spmm(int n3, const int32_t* __restrict__ ptr,
                                               const int32_t* __restrict__ col,
                                               const double4* __restrict__ val,
                                               const double* __restrict__ E,
                                               double* __restrict__ W) {
  const int r = blockIdx.x;
  const int lo = ptr[r], hi = ptr[r + 1];
  for (int nu = threadIdx.x; nu < n3; nu += 256) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = lo; k < hi; ++k) {
      const double e = E[(size_t)col[k] * n3 + nu];
      const double4 v = val[k];
      s0 += v.x * e;
      s1 += v.y * e;
      s2 += v.z * e;
    }
    W[((size_t)0 * n3 + r) * n3 + nu] = s0;
    W[((size_t)1 * n3 + r) * n3 + nu] = s1;
    W[((size_t)2 * n3 + r) * n3 + nu] = s2;
  }
}

constexpr int kQhTile = 64;
constexpr int kQhK = 16;

// One 64 x 64 tile of mode pairs (mu rows, nu columns, tile row <= tile
// column) per workgroup, four
// waves of 32 x 32: G_a = E^T W_a for a = x, y, z on v_mfma_f64_16x16x4f64
// (A[row = lane % 16][k = lane / 16], B[k = lane / 16][col = lane % 16];
// accumulator item r of lane l is row 4 r + l / 16, column l % 16), then per
// pair v_a = G_a/(2 sqrt(w_mu w_nu)) (the velocity matrix is -i G, and only
// the products G_a G_b enter), weight c tau, the six products, and
// tau |v|^2 per pair for the diffusivity, summed along each row in order.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void qh_gemm(
    int n3, int n_tiles, const double* __restrict__ E,
                                               const double* __restrict__ W,
                                               const double* __restrict__ omega,
                                               const double* __restrict__ gamma,
                                               const double4* __restrict__ mode, double hk,
                                               double* __restrict__ part,
                                               double* __restrict__ dpart) {
  constexpr int B = kQhTile, K = kQhK;
  constexpr int PER = K * B / 256;  // staged elements per thread and operand
  // the operand tiles during the K loop, the epilogue's row buffer after it
  __shared__ union {
    struct {
      double As[K][B];
      double Bs[3][K][B];
    } op;
    double Dp[B][B + 1];
  } sm;
  __shared__ double red[256][6];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // tiles ti <= tj only: G_a is antisymmetric, so every product G_a G_b and
  // the weights are symmetric in (mu, nu); an off-diagonal tile counts twice
  int ti = 0, k_rest = blockIdx.x;
  while (k_rest >= n_tiles - ti) {
    k_rest -= n_tiles - ti;
    ++ti;
  }
  const int tj = ti + k_rest;
  const int mu0 = ti * B, nu0 = tj * B;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const int lr = lane & 15, lg = lane >> 4;
  qd4 acc[3][2][2];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[a][x][y] = qd4{0.0, 0.0, 0.0, 0.0};
  // register staging of one K chunk: element e = tid + 256 u of the K x B
  // tile is (kk, cc) = (e / B, e % B)
  double ra[PER], rb[3][PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, kk = e / B, cc = e % B;
      const int c = k0 + kk;
      const bool in_k = c < n3;
      ra[u] = (in_k && mu0 + cc < n3) ? E[(size_t)c * n3 + mu0 + cc] : 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        rb[a][u] = (in_k && nu0 + cc < n3) ? W[((size_t)a * n3 + c) * n3 + nu0 + cc] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < n3; k0 += K) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, kk = e / B, cc = e % B;
      sm.op.As[kk][cc] = ra[u];
#pragma unroll
      for (int a = 0; a < 3; ++a) sm.op.Bs[a][kk][cc] = rb[a][u];
    }
    __syncthreads();
    if (k0 + K < n3) fetch(k0 + K);  // in flight during this chunk's products
#pragma unroll
    for (int kk = 0; kk < K; kk += 4) {
      double av[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = sm.op.As[kk + lg][wm + 16 * x + lr];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const double bv = sm.op.Bs[a][kk + lg][wn + 16 * y + lr];
#pragma unroll
          for (int x = 0; x < 2; ++x)
            acc[a][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv, acc[a][x][y], 0, 0, 0);
        }
    }
  }
  __syncthreads();  // the operand tiles are dead: Dp reuses their LDS
  // epilogue
  double kap[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int il = wm + 16 * x + 4 * r + lg, jl = wn + 16 * y + lr;
        const int mu = mu0 + il, nu = nu0 + jl;
        double dcontrib = 0.0;
        if (mu < n3 && nu < n3) {
          const double4 dm = mode[mu], dn = mode[nu];
          if (dm.w != 0.0 && dn.w != 0.0) {
            const double nrm = dm.z * dn.z;
            const double v0 = acc[0][x][y][r] * nrm, v1 = acc[1][x][y][r] * nrm,
                         v2 = acc[2][x][y][r] * nrm;
            const double w1 = omega[mu], w2 = omega[nu];
            const double tau = qh_pair_tau(w1, w2, gamma[mu], gamma[nu]);
            const double wt = qh_pair_c(w1, w2, dm.x, dn.x, dm.y, dn.y, hk) * tau;
            kap[0] += wt * v0 * v0;
            kap[1] += wt * v0 * v1;
            kap[2] += wt * v0 * v2;
            kap[3] += wt * v1 * v1;
            kap[4] += wt * v1 * v2;
            kap[5] += wt * v2 * v2;
            dcontrib = tau * (v0 * v0 + v1 * v1 + v2 * v2) * (1.0 / 3.0);
          }
        }
        sm.Dp[il][jl] = dcontrib;
      }
#pragma unroll
  for (int k = 0; k < 6; ++k) red[tid][k] = kap[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int k = 0; k < 6; ++k) red[tid][k] += red[tid + w][k];
    __syncthreads();
  }
  const double twice = ti == tj ? 1.0 : 2.0;
  if (tid < 6) part[(size_t)blockIdx.x * 6 + tid] = twice * red[0][tid];
  // diffusivity shares: row sums for the tile's mu (slot tj), and for an
  // off-diagonal tile the column sums for its nu (slot ti); every (slot,
  // mode) is written by exactly one tile
  if (dpart && tid < B) {
    double s = 0.0;
    for (int j = 0; j < B; ++j) s += sm.Dp[tid][j];
    if (mu0 + tid < n3) dpart[(size_t)tj * n3 + mu0 + tid] = s;
  } else if (dpart && ti != tj && tid < 2 * B) {
    const int jl = tid - B;
    double s = 0.0;
    for (int i = 0; i < B; ++i) s += sm.Dp[i][jl];
    if (nu0 + jl < n3) dpart[(size_t)ti * n3 + nu0 + jl] = s;
  }
}

// diffusivity[mu] = sum over the column tiles of the row partials, in order.
__global__ void qh_diff_finish(int n3, int n_tiles, const double* __restrict__ dpart,
                               double* __restrict__ diff) {
  const int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu >= n3) return;
  double s = 0.0;
  for (int t = 0; t < n_tiles; ++t) s += dpart[(size_t)t * n3 + mu];
  diff[mu] = s;
}

struct QhWs {
  size_t off_mode, off_part, off_cnt, off_ptr, off_col, off_val, off_frac, off_lat, off_w, off_dpart,
      total;
};

static QhWs qh_ws(long n_modes, long n_part, bool gamma_point, long n3) {
  QhWs w{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  w.off_mode = take(sizeof(double4) * n_modes);
  w.off_part = take(sizeof(double) * 6 * std::max<long>(1, n_part));
  if (gamma_point) {
    const int n_tiles = (int)((n3 + kQhTile - 1) / kQhTile);
    const long max_nnz = n3 * n3;  // bound before the count is known
    w.off_cnt = take(sizeof(int32_t) * n3);
    w.off_ptr = take(sizeof(int32_t) * (n3 + 1));
    w.off_col = take(sizeof(int32_t) * max_nnz);
    w.off_val = take(sizeof(double4) * max_nnz);
    w.off_frac = take(sizeof(double) * n3);
    w.off_lat = take(sizeof(double) * 9);
    w.off_w = take(sizeof(double) * 3 * n3 * n3);
    w.off_dpart = take(sizeof(double) * n_tiles * n3);
  }
  w.total = o;
  return w;
}

}  // namespace kaldo

using namespace kaldo;

extern "C" size_t kaldo_qhgk_crystal_workspace(const kaldo_crystal* c, const int32_t* mesh) {
  if (!c || !mesh || mesh[0] < 1 || mesh[1] < 1 || mesh[2] < 1) return 0;
  const long nq = (long)mesh[0] * mesh[1] * mesh[2];
  return qh_ws(nq * c->nb3, nq, false, 0).total;
}

extern "C" size_t kaldo_qhgk_gamma_workspace(const kaldo_crystal* c) {
  if (!c) return 0;
  const long n3 = c->nb3;
  const int n_tiles = (int)((n3 + kQhTile - 1) / kQhTile);
  return qh_ws(n3, (long)n_tiles * n_tiles, true, n3).total;
}

extern "C" int kaldo_qhgk_crystal(const kaldo_crystal* c, const int32_t* mesh, const double* frac,
                                  const double* omega, const double* evec, const double* gamma,
                                  double temperature, double nu_min_thz, void* workspace,
                                  size_t workspace_bytes, double* kappa, void* stream) {
  KALDO_REQUIRE(c && mesh && frac && omega && evec && gamma && kappa,
                "kaldo_qhgk_crystal: NULL argument");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "kaldo_qhgk_crystal: mesh must be >= 1");
  KALDO_REQUIRE(c->nb <= 5, "kaldo_qhgk_crystal: more than 5 basis atoms");
  KALDO_REQUIRE(std::isfinite(temperature) && temperature > 0, "kaldo_qhgk_crystal: temperature <= 0");
  KALDO_REQUIRE(std::isfinite(nu_min_thz) && nu_min_thz >= 0, "kaldo_qhgk_crystal: nu_min_thz < 0");
  for (int k = 0; k < 3 * c->nb; ++k)
    KALDO_REQUIRE(std::isfinite(frac[k]), "kaldo_qhgk_crystal: non-finite position");
  const long nq = (long)mesh[0] * mesh[1] * mesh[2];
  KALDO_REQUIRE(nq <= (1L << 30), "kaldo_qhgk_crystal: mesh too large");
  const QhWs w = qh_ws(nq * c->nb3, nq, false, 0);
  KALDO_REQUIRE(workspace && workspace_bytes >= w.total, "kaldo_qhgk_crystal: workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto* ws = static_cast<unsigned char*>(workspace);
  auto* mode = reinterpret_cast<double4*>(ws + w.off_mode);
  auto* part = reinterpret_cast<double*>(ws + w.off_part);
  QhCrystal p{};
  p.nq = (int)nq;
  p.nb3 = c->nb3;
  p.n_rep = c->n_rep;
  for (int k = 0; k < 3; ++k) p.N[k] = mesh[k];
  p.hk = kHbar / (kKb * temperature);
  for (int i = 0; i < c->nb; ++i)
    for (int a = 0; a < 3; ++a)
      p.tau_cart[i][a] = frac[3 * i] * c->lattice[a] + frac[3 * i + 1] * c->lattice[3 + a] +
                         frac[3 * i + 2] * c->lattice[6 + a];
  const long n_modes = nq * c->nb3;
  KALDO_LAUNCH("qh_modes", qh_modes, dim3(1), dim3(1024), 0, st, n_modes, omega, gamma, p.hk,
               nu_min_thz, mode, c->d_flags);
  const size_t lds = sizeof(double2) * std::max(1, c->n_rep);
#define KALDO_QH_CASE(NB3V)                                                                       \
  case NB3V:                                                                                      \
    KALDO_LAUNCH("qh_crystal", qh_crystal<NB3V>, dim3((unsigned)nq), dim3(256), lds, st, p,        \
                 c->d_fc2, c->d_repcart, c->d_rep, omega, gamma, evec, mode, part);               \
    break;
  switch (c->nb3) {
    KALDO_QH_CASE(3)
    KALDO_QH_CASE(6)
    KALDO_QH_CASE(9)
    KALDO_QH_CASE(12)
    KALDO_QH_CASE(15)
    default:
      set_error("kaldo_qhgk_crystal: unsupported branch count");
      return KALDO_EUNSUPPORTED;
  }
#undef KALDO_QH_CASE
  KALDO_LAUNCH("qh_finish", qh_finish, dim3(1), dim3(256), 0, st, nq, part,
               kKappaUnit / ((double)nq * c->volume), kappa);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}

extern "C" int kaldo_qhgk_gamma(const kaldo_crystal* c, const double* frac, const double* omega,
                                const double* evec, const double* gamma, double temperature,
                                double nu_min_thz, void* workspace, size_t workspace_bytes,
                                double* kappa, double* diffusivity, void* stream) {
  KALDO_REQUIRE(c && frac && omega && evec && gamma && kappa, "kaldo_qhgk_gamma: NULL argument");
  KALDO_REQUIRE(c->n_rep == 1, "kaldo_qhgk_gamma: the cell must have a single replica");
  KALDO_REQUIRE(std::isfinite(temperature) && temperature > 0, "kaldo_qhgk_gamma: temperature <= 0");
  KALDO_REQUIRE(std::isfinite(nu_min_thz) && nu_min_thz >= 0, "kaldo_qhgk_gamma: nu_min_thz < 0");
  for (int k = 0; k < 3 * c->nb; ++k)
    KALDO_REQUIRE(std::isfinite(frac[k]), "kaldo_qhgk_gamma: non-finite position");
  const int n3 = c->nb3;
  const int n_tiles = (n3 + kQhTile - 1) / kQhTile;
  const QhWs w = qh_ws(n3, (long)n_tiles * n_tiles, true, n3);
  KALDO_REQUIRE(workspace && workspace_bytes >= w.total, "kaldo_qhgk_gamma: workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto* ws = static_cast<unsigned char*>(workspace);
  auto* mode = reinterpret_cast<double4*>(ws + w.off_mode);
  auto* part = reinterpret_cast<double*>(ws + w.off_part);
  auto* cnt = reinterpret_cast<int32_t*>(ws + w.off_cnt);
  auto* ptr = reinterpret_cast<int32_t*>(ws + w.off_ptr);
  auto* col = reinterpret_cast<int32_t*>(ws + w.off_col);
  auto* val = reinterpret_cast<double4*>(ws + w.off_val);
  auto* dfrac = reinterpret_cast<double*>(ws + w.off_frac);
  auto* dlat = reinterpret_cast<double*>(ws + w.off_lat);
  auto* Wm = reinterpret_cast<double*>(ws + w.off_w);
  auto* dpart = reinterpret_cast<double*>(ws + w.off_dpart);
  // positions and cell into the workspace (host memory: a staged copy)
  KALDO_HIP(hipMemcpyAsync(dfrac, frac, sizeof(double) * 3 * c->nb, hipMemcpyHostToDevice, st));
  KALDO_HIP(hipMemcpyAsync(dlat, c->lattice, sizeof(double) * 9, hipMemcpyHostToDevice, st));
  const double hk = kHbar / (kKb * temperature);
  KALDO_LAUNCH("qh_modes", qh_modes, dim3(1), dim3(1024), 0, st, (long)n3, omega, gamma, hk,
               nu_min_thz, mode, c->d_flags);
  KALDO_LAUNCH("qh_csr_count", qh_csr_count, dim3(n3), dim3(64), 0, st, n3, c->d_fc2, cnt);
  KALDO_LAUNCH("qh_csr_scan", qh_csr_scan, dim3(1), dim3(1024), 0, st, n3, cnt, ptr);
  KALDO_LAUNCH("qh_csr_fill", qh_csr_fill, dim3(n3), dim3(64), 0, st, n3, c->d_fc2, dfrac, dlat, ptr,
               col, val);
  KALDO_LAUNCH("qh_spmm", qh_spmm, dim3(n3), dim3(256), 0, st, n3, ptr, col, val, evec, Wm);
  const int n_pairs = n_tiles * (n_tiles + 1) / 2;
  KALDO_LAUNCH("qh_gemm", qh_gemm, dim3(n_pairs), dim3(256), 0, st, n3, n_tiles, evec, Wm, omega,
               gamma, mode, hk, part, diffusivity ? dpart : nullptr);
  KALDO_LAUNCH("qh_finish", qh_finish, dim3(1), dim3(256), 0, st, (long)n_pairs, part,
               kKappaUnit / c->volume, kappa);
  if (diffusivity)
    KALDO_LAUNCH("qh_diff_finish", qh_diff_finish, dim3((n3 + 255) / 256), dim3(256), 0, st, n3,
                 n_tiles, dpart, diffusivity);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}
