// Shared host/device definitions of the linewidth library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/kaldo.h"

namespace kaldo {

// Physical constants (CODATA 2018) and unit conversions.
constexpr double kEvJ = 1.602176634e-19;     // J per eV
constexpr double kAmuKg = 1.66053906660e-27; // kg per amu
constexpr double kHbarJs = 1.054571817e-34;  // J s
constexpr double kKbJK = 1.380649e-23;       // J/K
constexpr double kHbar = kHbarJs / kEvJ * 1e12;            // eV ps
constexpr double kKb = kKbJK / kEvJ;                       // eV/K
constexpr double kU = kEvJ / (1e-20 * kAmuKg) * 1e-24;     // eV/(A^2 amu) in ps^-2
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;
constexpr double kSqrtPi = 1.77245385090551602730;
// W/(m K) per [k_B (A/ps)^2 ps / A^3]
constexpr double kKappaUnit = kKbJK * 1e4 * 1e-12 / 1e-30;
// Degenerate-cluster tolerance and velocity floor of the phonon solver (THz).
constexpr double kDegTolThz = 1e-4;
constexpr double kNuVelFloorThz = 1e-3;
// Modes with Gamma <= kGammaFloorRel * max Gamma carry no RTA conductivity.
constexpr double kGammaFloorRel = 1e-8;

constexpr int kMaxNb3Phonons = 32;
constexpr int kMaxNb3Linewidths = 16;

// Sticky device status of a handle (read and cleared by kaldo_device_status):
// bits the kernels set when they find a problem in device-resident inputs,
// with an atomic OR on the handle's status word (only on the error path).
constexpr int32_t kFlagNonFinite = 1;    // non-finite omega, eta, v or Gamma input
constexpr int32_t kFlagImaginary = 2;    // omega < 0 with |nu| >= nu_min
constexpr int32_t kFlagNoConverge = 4;   // an eigen-solver stopped at its sweep cap
constexpr int32_t kFlagSubset = 8;       // a modes_subset index outside [0, n_modes)
constexpr int32_t kFlagSingular = 16;    // a zero pivot in an LU factorisation
constexpr int32_t kFlagCache = 32;       // a temperature-cache row or pair index out of range
__device__ __forceinline__ void raise_flag(int32_t* flags, int32_t bit) { atomicOr(flags, bit); }

// ----------------------------------------------------------------- errors
void set_error(const std::string& msg);

#define KALDO_HIP(call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::kaldo::set_error(std::string(#call) + ": " + hipGetErrorString(e_));   \
      return KALDO_EDEVICE;                                                    \
    }                                                                          \
  } while (0)

#define KALDO_REQUIRE(cond, msg)                                               \
  do {                                                                         \
    if (!(cond)) {                                                             \
      ::kaldo::set_error(msg);                                                 \
      return KALDO_EINVAL;                                                     \
    }                                                                          \
  } while (0)

// ----------------------------------------------------------------- handle
// Crystal FC3 tables for the Bloch path, folded by d = l' - l'':
//   A~_q[e][s] = sum_{t in e} coef_t eta_{i_t}(q, s) e^{+i q.R_{l''_t}}
// with coef_t = Phi3_t / sqrt(m_i m_j m_k); entries e are sorted by d, and
// within a d by (jc, kc).  Then for q1 and q2 = -q - q1
//   V(q s; q1 s'; q2 s'') = sum_d e^{-i q1.R_d} sum_{e in d}
//                           A~_q[e][s] eta_{jc_e}(q1, s') eta_{kc_e}(q2, s'').
struct Fc3Bloch {
  int n_d = 0, n_e = 0, n_t = 0;
  int32_t* dvec = nullptr;   // [n_d][3]
  int32_t* d_ptr = nullptr;  // [n_d + 1] entry ranges
  int32_t* e_jc = nullptr;   // [n_e]
  int32_t* e_kc = nullptr;   // [n_e]
  int32_t* t_ptr = nullptr;  // [n_e + 1] contribution ranges
  int32_t* t_i = nullptr;    // [n_t] home-cell dof
  int32_t* t_l2 = nullptr;   // [n_t] replica index of the third index
  double* t_coef = nullptr;  // [n_t]
  // Atom-block view of the same entries: block = (jb, kb, d) with its 3x3
  // Cartesian (beta, gamma) sub-block; blocks sorted by (jb, kb, d).
  int n_blk = 0;
  int sym_jk = 0;               // Phi3(i, j, k) == Phi3(i, k, j) for every entry
  int32_t* e_blk = nullptr;     // [n_e] block of entry e
  int32_t* e_bg = nullptr;      // [n_e] 3*beta + gamma of entry e
  int32_t* blk_d = nullptr;     // [n_blk] d index of each block
  int32_t* pair_ptr = nullptr;  // [N_b*N_b + 1] block ranges per (jb, kb)
  // Work list for building one 16x16 B_s tile with a wave (3N_b <= 16):
  // slot k of lane l is entry k*64 + l of the (jc, kc) entries sorted by
  // their block count; int4 = (jc*17 + kc or -1, first block, end block, bg).
  int4* bwork = nullptr;        // [4][64]
};

// Gamma-point FC3: CSR over the (b, c) pattern of A_mu[b][c],
//   A_mu[b][c] = sum_{t in (b,c)} coef_t E[a_t][mu].
struct Fc3Gamma {
  int n_bc = 0, n_t = 0;
  int32_t* row_ptr = nullptr;  // [nb3 + 1] pattern ranges per row b
  int32_t* col = nullptr;      // [n_bc] column c of each pattern entry
  int32_t* t_ptr = nullptr;    // [n_bc + 1]
  int32_t* t_a = nullptr;      // [n_t]
  double* t_coef = nullptr;    // [n_t]
  // Row tiles of kSpmmRows rows of A_mu: the sorted unique columns each tile
  // touches (so a tile's E rows can be staged once in LDS), and the entries
  // in ELL form: slot t of row b (t < max_row) holds the row's t-th entry,
  // the position of its column in its tile's list at col_ell[t * nb3 + b]
  // (0 for the zero padding of shorter rows).
  int n_rtiles = 0, max_u = 0, max_tile_entries = 0, max_row = 0;
  int32_t* tile_u_ptr = nullptr;  // [n_rtiles + 1]
  int32_t* tile_u = nullptr;      // unique columns, concatenated
  int32_t* col_ell = nullptr;     // [max_row][nb3]
};
constexpr int kSpmmRows = 64;

}  // namespace kaldo

struct kaldo_crystal_s {
  int nb = 0, nb3 = 0, n_rep = 0;
  double lattice[9];
  double volume = 0.0;
  std::vector<double> mass;
  std::vector<int32_t> rep;
  std::vector<double> fc2;  // host copy, [nb3][n_rep][nb3]
  double* d_fc2 = nullptr;  // [nb3][n_rep][nb3] divided by sqrt(m m)
  int32_t* d_rep = nullptr; // [n_rep][3]
  double* d_repcart = nullptr;  // [n_rep][3] Cartesian replica vectors
  int32_t* d_flags = nullptr;   // sticky device status word (kFlag* bits)
  kaldo::Fc3Bloch bloch;
  kaldo::Fc3Gamma gamma;
  std::vector<void*> allocations;
};

namespace kaldo {
// Reciprocal rows b_c (with 2 pi) of a lattice given by rows a_i.
void reciprocal(const double* lattice, double* recip);

// Per-kernel event timing (see kaldo_profile_begin).
bool prof_on();
void prof_mark(const char* name, hipStream_t st, bool start);
}  // namespace kaldo

// Launch a kernel, bracketed by timing events when profiling is enabled.
#define KALDO_LAUNCH(name, kernel, grid, block, shmem, stream, ...)            \
  do {                                                                         \
    const bool p_ = ::kaldo::prof_on();                                        \
    if (p_) ::kaldo::prof_mark(name, stream, true);                            \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);       \
    if (p_) ::kaldo::prof_mark(name, stream, false);                           \
  } while (0)
