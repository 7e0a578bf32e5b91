// RTA thermal conductivity (paper: Eq. heatcap, Eq. rta; lifetime
// tau = 1/(2 Gamma) of Eq. lifetime).  One workgroup of 1024 threads (the
// call has no workspace for partial sums), fixed-order reduction.
#include <cmath>

#include "common.h"

namespace kaldo {

constexpr int kKappaThreads = 1024;

__global__ __launch_bounds__(kKappaThreads) void kappa_kernel(long n_modes, const double* __restrict__ omega,
                                                    const double* __restrict__ vel,
                                                    const double* __restrict__ gamma,
                                                    double inv_kt_hbar, double nu_min,
                                                    double scale, double* __restrict__ kappa,
                                                    int32_t* __restrict__ flags) {
  __shared__ double red[kKappaThreads][6];
  const int t = threadIdx.x;
  // max Gamma (order-independent)
  double gmax = 0.0;
  double chk = 0.0;  // x - x: 0 for finite inputs, NaN otherwise
  bool imag = false;
  for (long m = t; m < n_modes; m += kKappaThreads) {
    const double g = gamma[m], w = omega[m];
    gmax = fmax(gmax, g);
    chk += (g - g) + (w - w) + (vel[3 * m] - vel[3 * m]) + (vel[3 * m + 1] - vel[3 * m + 1]) +
           (vel[3 * m + 2] - vel[3 * m + 2]);
    imag = imag || (w < 0.0 && (-w / kTwoPi) >= nu_min);
  }
  if (!(chk == 0.0)) raise_flag(flags, kFlagNonFinite);
  if (imag) raise_flag(flags, kFlagImaginary);
  red[t][0] = gmax;
  __syncthreads();
  for (int w = kKappaThreads / 2; w > 0; w >>= 1) {
    if (t < w) red[t][0] = fmax(red[t][0], red[t + w][0]);
    __syncthreads();
  }
  const double floor_g = kGammaFloorRel * red[0][0];
  __syncthreads();
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long m = t; m < n_modes; m += kKappaThreads) {
    const double w = omega[m], g = gamma[m];
    if (!(w / kTwoPi >= nu_min) || !(g > floor_g) || !(g > 0.0)) continue;
    const double x = w * inv_kt_hbar;
    const double em = expm1(x);
    const double c = x * x * (em + 1.0) / (em * em);  // e^x = expm1(x) + 1
    const double ct = c * (1.0 / (2.0 * g));
    const double* v = vel + 3 * m;
    acc[0] += ct * v[0] * v[0];
    acc[1] += ct * v[0] * v[1];
    acc[2] += ct * v[0] * v[2];
    acc[3] += ct * v[1] * v[1];
    acc[4] += ct * v[1] * v[2];
    acc[5] += ct * v[2] * v[2];
  }
  for (int k = 0; k < 6; ++k) red[t][k] = acc[k];
  __syncthreads();
  for (int w = kKappaThreads / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int k = 0; k < 6; ++k) red[t][k] += red[t + w][k];
    __syncthreads();
  }
  if (t == 0) {
    const int map[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
    for (int k = 0; k < 9; ++k) kappa[k] = scale * red[0][map[k]];
  }
}

}  // namespace kaldo

using namespace kaldo;

extern "C" int kaldo_kappa_rta(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                               const double* vel, const double* gamma, double temperature,
                               double nu_min_thz, double* kappa, void* stream) {
  KALDO_REQUIRE(c && mesh && omega && vel && gamma && kappa, "kaldo_kappa_rta: NULL argument");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "kaldo_kappa_rta: mesh must be >= 1");
  KALDO_REQUIRE(std::isfinite(temperature) && temperature > 0, "kaldo_kappa_rta: temperature <= 0");
  KALDO_REQUIRE(std::isfinite(nu_min_thz) && nu_min_thz >= 0, "kaldo_kappa_rta: nu_min_thz < 0");
  const long nq = (long)mesh[0] * mesh[1] * mesh[2];
  const long n_modes = nq * c->nb3;
  const double scale = kKappaUnit / ((double)nq * c->volume);
  KALDO_LAUNCH("kappa_kernel", kappa_kernel, dim3(1), dim3(kKappaThreads), 0, static_cast<hipStream_t>(stream), n_modes,
                     omega, vel, gamma, kHbar / (kKb * temperature), nu_min_thz, scale, kappa, c->d_flags);
  KALDO_HIP(hipGetLastError());
  return KALDO_OK;
}
