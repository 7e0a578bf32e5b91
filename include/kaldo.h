/*
 * kaldo.h -- C ABI of the MI355X (gfx950) three-phonon linewidth library.
 *
 * The library computes, on one GPU, the hot path of anharmonic lattice
 * dynamics described in the kALDo 2.0 paper (arXiv 2602.23728):
 *
 *   phonons     harmonic frequencies, eigenvectors and group velocities from
 *               second-order force constants (paper: Eq. dynmat,
 *               Eq. dynmat_reciprocal, Eq. eigenvalue_crystal, Eq. groupvel);
 *   linewidths  three-phonon linewidths Gamma(q,s) from the sparse (COO)
 *               third-order force constants projected on three eigenvectors
 *               with Bloch phases, squared, and summed against Bose-Einstein
 *               populations and a smeared energy delta (Eq. phi3_proj,
 *               Eq. gamma with its Delta terms, Eq. broadening, Eq. bose,
 *               Eq. lifetime; the "Computational Implementation" list);
 *   kappa_rta   the RTA thermal conductivity tensor (Eq. heatcap, Eq. rta).
 *
 * Conventions shared by every call
 * --------------------------------
 * Units in: eV, Angstrom, amu, K.  Units out: omega and Gamma in rad/ps,
 * velocities in Angstrom/ps, kappa in W/(m K).  Cyclic widths (THz) are
 * converted with omega = 2 pi nu.
 *
 * Modes: mu = (q, s).  The q-mesh is Gamma-centred, q_n = sum_c (n_c/N_c) b_c,
 * flattened in C order over (n1, n2, n3): q = (n1*N2 + n2)*N3 + n3.  With
 * N_b basis atoms, nb3 = 3 N_b branches.
 *
 * Memory: every array argument documented "device" is a pointer into HBM of
 * the current HIP device (e.g. a torch CUDA tensor's data_ptr()); "host"
 * arguments are ordinary CPU memory read during the call only.  The library
 * keeps no pointer to caller memory past the call (or, for enqueued work,
 * past completion of that work on the caller's stream).  Device work is
 * enqueued on the caller's stream (hipStream_t passed as void*; NULL = the
 * legacy default stream) and the call returns after enqueueing; results are
 * valid after the stream is synchronised.
 *
 * Errors: every call returns a kaldo_status; no exception crosses the ABI.
 * Host arguments (sizes, structs, host arrays) are validated before anything
 * is enqueued (KALDO_EINVAL); device-runtime failures return KALDO_EDEVICE.
 * Device-resident inputs cannot be read before the call returns without a
 * synchronisation, so the kernels validate them as they read them and record
 * what they find in a sticky status word of the crystal handle:
 * kaldo_device_status() synchronises the stream, returns that status
 * (KALDO_EINVAL for a non-finite omega/eta/v/Gamma, a subset index or a
 * temperature-cache index out of range, KALDO_ENUMERIC for an imaginary mode above nu_min or an eigen-solver
 * that stopped at its sweep cap) and clears it.  kaldo_last_error() returns
 * a thread-local description of the last failure in the calling thread.
 *
 * Determinism: all reductions run in a fixed order; identical inputs give
 * bit-identical outputs.
 */
#ifndef KALDO_H
#define KALDO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KALDO_OK = 0,
  KALDO_EINVAL = -1,      /* bad argument: shape, range, NULL, NaN        */
  KALDO_ENOMEM = -2,      /* allocation failed (handle creation only)     */
  KALDO_EDEVICE = -3,     /* HIP runtime error                            */
  KALDO_ENUMERIC = -4,    /* numerical failure (e.g. no eigen convergence)*/
  KALDO_EUNSUPPORTED = -5 /* valid request the library does not implement */
} kaldo_status;

/* Arithmetic of the vertex contraction (projection of Phi3 on eigenvectors).
 * Frequencies, widths, the 2-sigma cut, populations, |V|^2 weights and all
 * accumulations are FP64 in every mode. */
typedef enum {
  KALDO_FP64 = 0,   /* contraction in FP64                                  */
  KALDO_FP32 = 1,   /* operands rounded to FP32, FP32 products and sums     */
  KALDO_BF16X3 = 2  /* operands split x = hi + lo (bf16 each); products
                       hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32 accumulation;
                       cells of fewer than 9 branches run the FP32 form
                       instead (the 16-wide matrix-core tiles would be mostly
                       padding: the pruned FP32 kernel is faster there and at
                       least as accurate) */
} kaldo_precision;

typedef enum { KALDO_GAUSS = 0, KALDO_LORENTZ = 1 } kaldo_shape;

/* Energy-conservation smearing (paper: Eq. broadening and the text after it).
 * shape      Gaussian exp(-x^2/s^2)/(sqrt(pi) s) or Lorentzian
 *            (s/2)/(pi (x^2 + s^2/4)); both are 0 unless |x| < 2 s.
 * adaptive   0: s = 2 pi sigma_thz.  1: per scattering pair
 *            s = max(2 pi sigma_floor_thz, |dv| h / sqrt(12)), with h^2 the
 *            mean of |b_c/N_c|^2 over the three mesh axes and dv the velocity
 *            difference of the two partner phonons of that process.
 * nu_min_thz modes with cyclic frequency below it get Gamma = 0 and take no
 *            part as scattering partners (the paper's min_frequency).       */
typedef struct {
  int32_t shape;
  int32_t adaptive;
  double sigma_thz;
  double sigma_floor_thz;
  double nu_min_thz;
} kaldo_broadening;

/* Opaque handle: one crystal (or one Gamma-point cell) with its force
 * constants resident in device memory. */
typedef struct kaldo_crystal_s kaldo_crystal;

/* kaldo_crystal_create -- upload a cell and its force constants.
 * (paper: "Interatomic Force Constants": FC2 dense 3N_b x 3N, FC3 sparse COO
 *  3N_b x (3N)^2 with the first index in the home cell.)
 *   n_basis     N_b >= 1
 *   lattice     host double[9], rows a1, a2, a3 in Angstrom
 *   mass        host double[N_b], amu, > 0
 *   n_rep       number of replicas (cells) the FCs reach, >= 1
 *   rep         host int32[n_rep][3] integer replica coordinates, rep[0] must
 *               be (0,0,0) (a Gamma-point solid passes n_rep = 1)
 *   fc2         host double[3N_b][n_rep][3N_b], eV/A^2:
 *               fc2[3i+a][l][3j+b] = Phi(0 i a, l j b)
 *   nnz, fc3_i, fc3_j, fc3_k, fc3_val
 *               host COO: fc3_i in [0, 3N_b) is 3*basis+alpha of the home
 *               atom; fc3_j, fc3_k in [0, 3 N_b n_rep) are
 *               (rep*N_b + basis)*3 + beta; values eV/A^3.  Any order;
 *               duplicates are summed.
 *   out         receives the handle.
 * Allocates device memory on the current device (KALDO_ENOMEM on failure);
 * the handle owns it until kaldo_crystal_destroy.  Synchronous. */
int kaldo_crystal_create(int32_t n_basis, const double* lattice, const double* mass,
                         int32_t n_rep, const int32_t* rep, const double* fc2,
                         int64_t nnz, const int32_t* fc3_i, const int32_t* fc3_j,
                         const int32_t* fc3_k, const double* fc3_val,
                         kaldo_crystal** out);

/* Frees the handle and its device memory.  NULL is a no-op.  Synchronous
 * (hipFree); call it before the process starts tearing down the HIP runtime,
 * not from a static destructor or an interpreter finaliser. */
int kaldo_crystal_destroy(kaldo_crystal* c);

/* kaldo_device_status -- outcome of the device-side input checks of every
 * call made on this handle since the last query (paper: the selective
 * calculation of "Computational Implementation", whose min_frequency makes a
 * mode below it unphysical; a mode with omega^2 < 0 above it is an error).
 * Synchronises `stream` (the stream the calls were enqueued on), reads the
 * handle's status word and clears it.  Returns KALDO_OK if nothing was found;
 * KALDO_EINVAL if a kernel read a non-finite omega, eigenvector component,
 * velocity or linewidth, a modes_subset index outside [0, n_modes), or a
 * temperature-cache row pointer or partner index out of range (such entries
 * are ignored); KALDO_ENUMERIC if a mode had omega < 0 with
 * |nu| >= nu_min_thz (the linewidth and conductivity kernels treat it as
 * unphysical), if kaldo_phonons' Jacobi solver reached its sweep cap on
 * some q, or if kaldo_bte_solve met a zero pivot.  kaldo_last_error() then lists every condition found.  Calls on
 * other streams that are still running may set the word after it is read. */
int kaldo_device_status(kaldo_crystal* c, void* stream);

/* kaldo_phonons -- harmonic phonons on a Gamma-centred mesh, FP64 on the GPU.
 * (paper: Eq. dynmat_reciprocal with phase e^{-i q.R_l}, Eq. eigenvalue_crystal,
 *  Eq. groupvel with the analytic dD/dq.)  One Hermitian eigenproblem per q.
 *   mesh    host int32[3], each >= 1
 *   omega   device double[N_q][nb3]   rad/ps, ascending per q;
 *           omega = sign(lambda) sqrt(|lambda|) for eigenvalue lambda of D
 *   evec    device double[N_q][nb3][nb3][2] complex, [q][component][mode]:
 *           unit columns; within a cluster of frequencies closer than
 *           1e-4 THz the basis diagonalises sum_c chat_c dD/dq_c with
 *           chat = (1,2,3)/sqrt(14); each column's largest-modulus component
 *           is real positive
 *   vel     device double[N_q][nb3][3]  Angstrom/ps, diagonal Hellmann-Feynman
 *           elements; 0 where |nu| < 1e-3 THz
 * Requires nb3 <= 32 (one workgroup per q, matrices held in LDS); larger
 * cells at the Gamma point use kaldo_phonons_gamma.  Cyclic Jacobi, at most
 * 60 sweeps (converged to off-diagonal norm <= 1e-16 of the total); a q whose
 * solver stops at the cap sets the handle's non-convergence status
 * (kaldo_device_status -> KALDO_ENUMERIC).  The environment variable
 * KALDO_JACOBI_SWEEPS (1..60) lowers the cap, for tests of that status. */
int kaldo_phonons(const kaldo_crystal* c, const int32_t* mesh, double* omega,
                  double* evec, double* vel, void* stream);

/* kaldo_phonons_gamma -- Gamma-point phonons of one cell: the real symmetric
 * D = sum_l Phi(0, l)/sqrt(m m) (paper: Eq. dynmat, Eq. eigenvalue),
 * diagonalised in FP64 on the host (Householder tridiagonalisation and the
 * implicit QL method).  Synchronous; needs no GPU.
 *   n_basis, mass, n_rep, fc2   host, layouts of kaldo_crystal_create
 *   omega   host double[nb3] rad/ps ascending, sign(lambda) sqrt(|lambda|)
 *   evec    host double[nb3][nb3] real, [component][mode], unit columns, each
 *           column's largest-modulus component positive
 * KALDO_ENUMERIC if the QL iteration does not converge. */
int kaldo_phonons_gamma(int32_t n_basis, const double* mass, int32_t n_rep, const double* fc2,
                        double* omega, double* evec);

/* Device workspace bytes kaldo_linewidths needs for this crystal, mesh and
 * precision. */
size_t kaldo_linewidths_workspace(const kaldo_crystal* c, const int32_t* mesh,
                                  int32_t precision);

/* kaldo_linewidths -- three-phonon linewidths of a crystal on a mesh.
 * (paper: Eq. phi3_proj with Bloch phases, all-incoming momenta
 *  q + q1 + q2 = G; Eq. gamma with populations paired as
 *  coalescence (n1 - n2) delta(w + w1 - w2) and decay
 *  1/2 (n1 + n2 + 1) delta(w - w1 - w2); 1/N_q Bloch normalisation;
 *  Eq. broadening with the |x| < 2 sigma cut; Eq. bose.)
 *   Gamma(q,s) = pi hbar U^3/(8 N_q) sum_{q1,s',s''} m |V|^2/(w w1 w2)
 *                [(n1 - n2) g(x+) + 1/2 (n1 + n2 + 1) g(x-)]
 *   with x+ = (w + w1) - w2, x- = (w - w1) - w2 in FP64, q2 = -q - q1.
 *   mesh           host int32[3]
 *   omega, evec, vel   device, layouts of kaldo_phonons
 *   temperature    K, > 0
 *   broadening     host struct
 *   precision      kaldo_precision
 *   modes_subset   device int32[n_subset] flat mode indices q*nb3 + s, or NULL
 *                  for all modes; only those entries of gamma are written
 *   workspace      device buffer of kaldo_linewidths_workspace() bytes
 *   gamma          device double[N_q*nb3] rad/ps
 * Requires nb3 <= 16. */
int kaldo_linewidths(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                     const double* evec, const double* vel, double temperature,
                     const kaldo_broadening* broadening, int32_t precision,
                     const int32_t* modes_subset, int64_t n_subset, void* workspace,
                     size_t workspace_bytes, double* gamma, void* stream);

/* kaldo_linewidths_noalloc -- kaldo_linewidths without a workspace argument
 * and without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and kernels as kaldo_linewidths; the
 * workspace is a device array inside the library, one per GPU, of
 * kaldo_linewidths_noalloc_max_bytes() bytes (32 MiB), held until the process
 * ends.  A request whose kaldo_linewidths_workspace() exceeds that size
 * returns KALDO_EINVAL before anything is enqueued.  Every call on one GPU
 * uses that GPU's array: calls that overlap in time on one GPU (other streams,
 * other threads) race and must be serialised by the caller; nothing needs
 * clearing between calls (every byte read is written first within a call). */
int kaldo_linewidths_noalloc(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                             const double* evec, const double* vel, double temperature,
                             const kaldo_broadening* broadening, int32_t precision,
                             const int32_t* modes_subset, int64_t n_subset, double* gamma,
                             void* stream);

/* Size in bytes of kaldo_linewidths_noalloc's device scratch array. */
size_t kaldo_linewidths_noalloc_max_bytes(void);

/* Device workspace bytes kaldo_linewidths_gamma needs. */
size_t kaldo_linewidths_gamma_workspace(const kaldo_crystal* c, int32_t precision);

/* kaldo_linewidths_gamma -- linewidths of a Gamma-point solid (N_q = 1, real
 * eigenvectors): V_mu = E^T A_mu E with A_mu[b][c] = sum_a Phi3_abc E_a,mu /
 * sqrt(m_a m_b m_c); same rate formula with N_q = 1 and fixed-width smearing
 * (paper: Eq. phi3_proj, Eq. gamma; the Gamma-point QHGK setting).
 *   omega       device double[nb3] rad/ps
 *   evec        device double[nb3][nb3] real [component][mode]
 *   modes_subset device int32[n_subset] or NULL
 *   gamma       device double[nb3]
 * broadening->adaptive must be 0. */
int kaldo_linewidths_gamma(const kaldo_crystal* c, const double* omega, const double* evec,
                           double temperature, const kaldo_broadening* broadening,
                           int32_t precision, const int32_t* modes_subset, int64_t n_subset,
                           void* workspace, size_t workspace_bytes, double* gamma,
                           void* stream);

/* kaldo_kappa_rta -- RTA conductivity (paper: Eq. heatcap, Eq. rta, with
 * tau = 1/(2 Gamma) of Eq. lifetime):
 *   kappa_ab = 1/(N_q V_cell) sum_mu c_mu v_mu,a v_mu,b / (2 Gamma_mu)
 * over modes with nu >= nu_min_thz and Gamma_mu > 1e-8 max(Gamma).
 *   omega, vel, gamma  device, layouts of kaldo_phonons / kaldo_linewidths
 *   n_modes            N_q * nb3
 *   kappa              device double[9] W/(m K), row-major
 * Fixed-order single-workgroup reduction. */
int kaldo_kappa_rta(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                    const double* vel, const double* gamma, double temperature,
                    double nu_min_thz, double* kappa, void* stream);

/* ------------------------------------------------------------------------
 * Full linearised BTE (paper, "Boltzmann Transport Equation": Eq. BTE,
 * Eq. gamma1, Eq. invBTE, Eq. kappa_general, Eq. sc_iter, Eq. inverse).
 * The scattering matrix Gamma~ = diag(Gamma0) + Gamma1 over all
 * n = N_q nb3 modes (rad/ps, dense FP64, row-major, caller-owned device
 * buffer of n*n doubles), built from the same vertex, cut, widths and
 * populations as kaldo_linewidths (Gamma0 = 2 Gamma).  Per ordered candidate
 * (q s; q1 s'; q2 s'') with coalescence and decay rates
 *   d+ = 2 P |V|^2 (n1 - n2) g(x+)/(w w1 w2), d- = P |V|^2 (n1 + n2 + 1) g(x-)/(w w1 w2)
 * (P = pi hbar U^3/(8 N_q)), row (q, s) receives Gamma0 += d+ + d-,
 * column (q1, s') += d+ w1/w, column tr(q1, s') -= d- w1/w and column
 * tr(q2, s'') -= (d+ + d-) w2/w, where tr() is the time-reversal partner (the
 * mode at -q' whose eigenvector overlaps eta(q', s')* most).  These rows make
 * Eq. sc_iter the iterative scheme of the adaptive-smearing reference the
 * paper cites (the printed Eq. gamma1 is read this way).  Modes with
 * nu < nu_min or Gamma0 <= 1e-8 max Gamma0 are decoupled (zero row and
 * column, unit diagonal, lambda = 0).  Cells of 1 or 2 atoms
 * (KALDO_EUNSUPPORTED otherwise); N_q <= 65535.
 * ------------------------------------------------------------------------ */

/* Device workspace bytes of kaldo_scattering_matrix, kaldo_bte_solve and
 * kaldo_bte_iterate (one workspace serves all three). */
size_t kaldo_bte_workspace(const kaldo_crystal* c, const int32_t* mesh);

/* kaldo_scattering_matrix -- builds Gamma~ into `matrix` (device double[n][n])
 * and the diagonal rates Gamma0 into `gamma0` (device double[n]); FP64
 * projection, fixed-order sums (bitwise reproducible).
 *   omega, evec, vel, temperature, broadening: as kaldo_linewidths */
int kaldo_scattering_matrix(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                            const double* evec, const double* vel, double temperature,
                            const kaldo_broadening* broadening, void* workspace,
                            size_t workspace_bytes, double* matrix, double* gamma0, void* stream);

/* kaldo_bte_solve -- Eq. inverse: lambda = Gamma~^-1 v (device double[n][3],
 * Angstrom) by a blocked LU factorisation without pivoting (64 x 64 blocks,
 * trailing updates on the FP64 matrix cores), then
 * kappa_ab = 1/(N_q V) sum c v_a lambda_b (device double[9], W/(m K)).
 * The decoupled modes (see above: lambda = 0) are left out of the
 * factorisation, which runs on the block of the coupled ones.  `matrix` is
 * overwritten: in each coupled row the coupled columns are moved to the
 * front and the coupled block's LU factors stored there; the decoupled rows
 * are untouched.  A zero pivot sets the handle's status (kaldo_device_status
 * -> KALDO_ENUMERIC).  Synchronises `stream` once (the number of coupled modes
 * sizes the factorisation); the rest is enqueued. */
int kaldo_bte_solve(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                    const double* vel, const double* gamma0, double temperature,
                    double nu_min_thz, double* matrix, void* workspace, size_t workspace_bytes,
                    double* lambda, double* kappa, void* stream);

/* kaldo_bte_iterate -- Eq. sc_iter from the RTA start lambda0 = v/Gamma0:
 * lambda <- (v - Gamma1 lambda)/Gamma0 until |k_new - k_old| <= tolerance
 * |k_old| for k = Tr(kappa)/3, or n_iterations updates.  `matrix` is read
 * only.  Synchronises `stream` once per iteration (the stopping test is on
 * the host); *iterations (host, may be NULL) = updates done.  Returns
 * KALDO_ENUMERIC if it did not stop within n_iterations (the iteration
 * contracts only when the off-diagonal part is small against the diagonal);
 * lambda and kappa then hold the last iterate. */
int kaldo_bte_iterate(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                      const double* vel, const double* gamma0, double temperature,
                      double nu_min_thz, const double* matrix, int32_t n_iterations,
                      double tolerance, void* workspace, size_t workspace_bytes, double* lambda,
                      double* kappa, int32_t* iterations, void* stream);

/* ------------------------------------------------------------------------
 * Isotope scattering, Eq. isotope (Tamura's perturbation theory, "Isotopic
 * Scattering"):
 *   gamma_iso(q,s) = pi/(2 N_q) w^2 sum_{q' s'} g(w - w'; sigma')
 *                    sum_i g_i |sum_a eta*_{ia}(q,s) eta_{ia}(q',s')|^2
 * The Cartesian sum sits inside the modulus (Tamura's form; it does not
 * depend on the orientation of the axes, the printed placement outside the
 * modulus would).  g(x; sigma) is the smearing of Eq. broadening with its
 * 2 sigma cut; partners and modes below nu_min are excluded; the adaptive
 * width of a partner is max(sigma_floor, |v(q',s')| h / sqrt(12)) (h^2 the
 * mean-square mesh step, as for kaldo_linewidths), the rate at which w - w'
 * varies with q'.  gamma_iso is a linewidth in the convention of Eq. gamma
 * (the paper adds the two; tau = 1/(2 Gamma), Eq. lifetime).
 * ------------------------------------------------------------------------ */

/* Device workspace bytes of kaldo_isotope_linewidths (0 on bad arguments). */
size_t kaldo_isotope_workspace(const kaldo_crystal* c, const int32_t* mesh);

/* kaldo_isotope_linewidths -- gamma_iso of every mode (crystal cells of at
 * most 5 basis atoms, else KALDO_EINVAL), FP64 throughout, fixed summation
 * order (bitwise reproducible).
 *   omega, evec, vel  device, layouts of kaldo_phonons
 *   g_factor          host double[n_basis]: g_i = sum_iso f (dM/M_i)^2 of
 *                     each basis atom, finite and >= 0 (the library knows
 *                     no isotope tables: the caller supplies them)
 *   broadening        shape, fixed or adaptive width, nu_min (as above)
 *   accumulate        0: gamma = gamma_iso; 1: gamma += gamma_iso (e.g. onto
 *                     the anharmonic Gamma of kaldo_linewidths)
 *   gamma             device double[N_q][3 N_b], rad/ps; modes below nu_min
 *                     get 0 (accumulate 0) or are left as they are
 * Non-finite omega, eta or v and imaginary modes above nu_min set the
 * handle's status word (kaldo_device_status).  Enqueued; returns at once. */
int kaldo_isotope_linewidths(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                             const double* evec, const double* vel, const double* g_factor,
                             const kaldo_broadening* broadening, int32_t accumulate,
                             void* workspace, size_t workspace_bytes, double* gamma,
                             void* stream);

/* ------------------------------------------------------------------------
 * Quasi-harmonic Green-Kubo conductivity ("Quasi-Harmonic Green-Kubo"):
 *   kappa_ab = 1/V sum_{mu nu} c_{mu nu} v^a_{mu nu} tau_{mu nu} v^b_{nu mu}
 * (Eq. qhgk for a Gamma-point solid; for a crystal the s != s' pairs of each
 * q, the interband term of Eq. qhgk_crystal, which adds to kaldo_kappa_rta's
 * result).  Readings: c_{mu nu} = (hbar/T) w_mu w_nu (n_mu - n_nu)/(w_nu -
 * w_mu) (the printed prefactor k_B/T would not reduce to Eq. heatcap's c_mu
 * for w_nu -> w_mu; pairs closer than 1e-4 THz take the mean c); v^a_{mu nu}
 * = eta_mu^H (dD/dq_a) eta_nu / (2 sqrt(w_mu w_nu)) with dD/dq_a built from
 * the full separation of the two atoms (lattice vector plus basis offset, the
 * minimum image within one cell), whose diagonal is the group velocity;
 * tau_{mu nu} = g/(2((w_mu - w_nu)^2 + g^2)) with g = (Gamma_mu +
 * Gamma_nu)/2 (Lorentzian, as printed), so tau_{mu mu} = 1/(2 Gamma_mu).
 * Modes taken: nu >= nu_min and Gamma > 1e-8 max Gamma (as kaldo_kappa_rta).
 * V: N_q times the cell volume.  FP64, fixed summation order.
 * ------------------------------------------------------------------------ */

/* Device workspace bytes of kaldo_qhgk_crystal / kaldo_qhgk_gamma. */
size_t kaldo_qhgk_crystal_workspace(const kaldo_crystal* c, const int32_t* mesh);
size_t kaldo_qhgk_gamma_workspace(const kaldo_crystal* c);

/* kaldo_qhgk_crystal -- the interband term of Eq. qhgk_crystal (cells of at
 * most 5 basis atoms).
 *   frac              host double[n_basis][3] fractional basis positions
 *                     (the handle keeps none; needed for the separations)
 *   omega, evec       device, layouts of kaldo_phonons
 *   gamma             device double[N_q][nb3] linewidths (rad/ps)
 *   kappa             device double[9] out, W/(m K)
 * Non-finite omega or Gamma and imaginary modes above nu_min set the handle's
 * status word.  Enqueued; returns at once. */
int kaldo_qhgk_crystal(const kaldo_crystal* c, const int32_t* mesh, const double* frac,
                       const double* omega, const double* evec, const double* gamma,
                       double temperature, double nu_min_thz, void* workspace,
                       size_t workspace_bytes, double* kappa, void* stream);

/* kaldo_qhgk_gamma -- Eq. qhgk for a Gamma-point solid (a handle with one
 * replica), on the FP64 matrix cores.
 *   frac              host double[n_basis][3] fractional positions, copied to
 *                     the workspace on `stream`
 *   omega, evec       device, layouts of kaldo_linewidths_gamma (real E)
 *   gamma             device double[nb3] linewidths (rad/ps)
 *   kappa             device double[9] out, W/(m K)
 *   diffusivity       device double[nb3] out or NULL: D_mu = 1/3 sum_a sum_nu
 *                     |v^a_{mu nu}|^2 tau_{mu nu} (A^2/ps), 0 for modes not taken
 * Each bonded pair must have a single image within the force-constant range
 * (minimum-image separations).  Enqueued; returns at once. */
int kaldo_qhgk_gamma(const kaldo_crystal* c, const double* frac, const double* omega,
                     const double* evec, const double* gamma, double temperature,
                     double nu_min_thz, void* workspace, size_t workspace_bytes, double* kappa,
                     double* diffusivity, void* stream);

/* ------------------------------------------------------------------------
 * Temperature sweeps.  The paper separates the temperature-invariant part of
 * the calculation from the populations so that a sweep over temperatures
 * reuses the projection of Eq. phi3_proj ("Performance and Scalability",
 * multi-temperature optimisation).  In Eq. gamma only the Bose populations of
 * the two partners (Eq. bose) depend on T, so the library stores, per mode
 * and per partner entry that passes the 2-sigma cut, two factors c and d with
 *   Gamma_mu(T) = pi hbar U^3/(8 N_q) sum_row c (n1 - n2) + d (n1 + n2 + 1),
 *   c = |V|^2 g(x+)/(w w1 w2),  d = 1/2 |V|^2 g(x-)/(w w1 w2)
 * (each g zero outside its cut).  When Phi3 is symmetric in its last two
 * slots one entry stands for a pair and its mirror (q2 s'', q1 s'): then
 * c = |V|^2 (g(x+) - g(x+')) / (w w1 w2) and d sums both decay terms, x+' =
 * (w + w2) - w1.
 * ------------------------------------------------------------------------ */

/* Device workspace bytes of kaldo_tcache_build (0 on bad arguments). */
size_t kaldo_tcache_workspace(const kaldo_crystal* c, const int32_t* mesh, int32_t precision);

/* kaldo_tcache_build -- the temperature-independent factors of every mode in
 * modes_subset (all modes when modes_subset is NULL), computed by the fused
 * pruned kernel (cells of at most 5 basis atoms and 64 replicas whose A~
 * tables fit in LDS; else KALDO_EUNSUPPORTED; precision FP64 or FP32 for the
 * projection, factors always FP64).  Rows are CSR by mode:
 *   row_ptr    device int64[n_modes + 1] out: entries of mode m are
 *              [row_ptr[m], row_ptr[m+1]); rows of modes not selected or
 *              below nu_min are empty
 *   capacity   entries `pairs` and `factors` can hold
 *   pairs      device uint32[capacity][2] out: flat partner modes (m1, m2)
 *   factors    device double[capacity][2] out: (c, d) as above
 *   n_entries  host out: entries needed
 * Runs a count pass, writes row_ptr and synchronises `stream` once to read
 * the total.  With pairs and factors NULL it stops there (a size query);
 * with capacity < *n_entries it returns KALDO_EINVAL and writes no entry;
 * otherwise a record pass fills the rows (enqueued; valid after a stream
 * synchronisation).  The order of a row is fixed by the inputs, so the
 * output is bitwise reproducible.  Other arguments as kaldo_linewidths. */
int kaldo_tcache_build(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                       const double* evec, const double* vel, const kaldo_broadening* broadening,
                       int32_t precision, const int32_t* modes_subset, int64_t n_subset,
                       void* workspace, size_t workspace_bytes, int64_t* row_ptr, int64_t capacity,
                       uint32_t* pairs, double* factors, int64_t* n_entries, void* stream);

/* Device workspace bytes of kaldo_tcache_gamma (0 on bad arguments). */
size_t kaldo_tcache_gamma_workspace(const kaldo_crystal* c, const int32_t* mesh);

/* kaldo_tcache_gamma -- Gamma at each of n_temps temperatures (host
 * double[n_temps], K, finite and > 0) from a cache of kaldo_tcache_build:
 *   gamma   device double[n_temps][n_modes] out, rad/ps; 0 for modes below
 *           nu_min_thz and for empty rows
 * One pass over the entries per batch of up to 8 temperatures; FP64, fixed
 * summation order (bitwise reproducible).  Row pointers outside
 * [0, n_entries] or partner indices outside [0, n_modes) are skipped and set
 * the handle's status (kaldo_device_status -> KALDO_EINVAL).  Enqueued. */
int kaldo_tcache_gamma(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                       double nu_min_thz, const int64_t* row_ptr, int64_t n_entries,
                       const uint32_t* pairs, const double* factors, int32_t n_temps,
                       const double* temperatures, void* workspace, size_t workspace_bytes,
                       double* gamma, void* stream);

/* ------------------------------------------------------------------------
 * Learned form.  The paper restricts the scattering calculation to the
 * irreducible wedge of the mesh and maps the results back onto the full grid
 * (overview of the 2.0 computational changes), and lists the scattering
 * phase space among its computed quantities ("Phonon Properties and
 * Scattering"; no formula is given).  The MLP ensemble, its features and
 * the gate below are this library's own: no surrogate appears in the paper.
 * All device entry points enqueue on `stream` and return; results are valid
 * after a stream synchronisation unless stated otherwise.
 * ------------------------------------------------------------------------ */

/* kaldo_mesh_ibz -- irreducible wedge of a Gamma-centred mesh (host, FP64).
 * Point operations are the integer matrices M (entries -1..1 in the lattice
 * basis) that keep the metric and map the basis onto itself (equal masses,
 * up to a translation); q and M^T q share a star when M^T q lies on the
 * mesh (non-cubic meshes keep the operations that do).  A reduced basis is
 * assumed (then every point operation has entries in -1..1).
 *   lattice    host double[3][3] rows a_i (Angstrom)
 *   frac       host double[n_basis][3] fractional positions
 *   mass       host double[n_basis] amu
 *   mesh       host int32[3]
 *   ir_of_q    host int32[N_q] out: the smallest flat index in the star of q
 *   star_size  host int32[N_q] out: star size at representatives, else 0
 *   n_ops_out, n_ir_out  host int32 out (may be NULL) */
int kaldo_mesh_ibz(const double* lattice, int32_t n_basis, const double* frac,
                   const double* mass, const int32_t* mesh, int32_t* ir_of_q,
                   int32_t* star_size, int32_t* n_ops_out, int32_t* n_ir_out);

/* Device workspace bytes kaldo_jdos needs (0 on bad arguments). */
size_t kaldo_jdos_workspace(const kaldo_crystal* c, const int32_t* mesh);

/* kaldo_jdos -- two-phonon joint density of states, read as the partner count
 * of Eq. gamma without the vertex and populations, with the same cut
 * |x| < 2 sigma, smearing, widths and nu_min masks as kaldo_linewidths:
 *   D+(q,s) = (1/N_q) sum_{q1 s' s''} m g((w + w1) - w2; sigma+)
 *   D-(q,s) = (1/N_q) sum_{q1 s' s''} m g((w - w1) - w2; sigma-)
 * with q2 = -q - q1 (mod G) and m = [nu1 >= nu_min][nu2 >= nu_min]; 0 for
 * modes below nu_min.  Units ps/rad.  Cut decisions and sums in FP64.
 *   omega, vel     device, layouts of kaldo_phonons
 *   modes_subset   device int32[n_subset] or NULL (all modes); only those
 *                  entries of dplus / dminus are written
 *   dplus, dminus  device double[N_q*nb3]
 * Requires nb3 <= 16 and N_q <= 65535 (KALDO_EINVAL otherwise).  Each
 * unordered partner pair {q1, q2} is visited once and contributes the terms
 * of both orderings, each with its own cut; sums are in a fixed order, so
 * results are bitwise reproducible. */
int kaldo_jdos(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
               const double* vel, const kaldo_broadening* broadening,
               const int32_t* modes_subset, int64_t n_subset, void* workspace,
               size_t workspace_bytes, double* dplus, double* dminus, void* stream);

/* Feature count per row: nb3 + 8 (at most 32). */
int32_t kaldo_surrogate_feature_count(const kaldo_crystal* c);

/* kaldo_surrogate_features -- row k for mode m = modes[k] (float32):
 *   nu (THz), |v| (A/ps), one-hot branch (nb3 entries), the ascending
 *   |components| of the shortest Cartesian image q + G (1/A), |q + G|,
 *   ln(1 + D+), ln(1 + D-).
 *   modes     device int32[n] flat mode indices
 *   features  device float[n][nb3 + 8] */
int kaldo_surrogate_features(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                             const double* vel, const double* dplus, const double* dminus,
                             const int32_t* modes, int64_t n, float* features, void* stream);

/* kaldo_standardize -- column means and population standard deviations over
 * the first n_fit rows (FP64), then every row of X (device float[n][n_feat])
 * standardised in place; sd = 1 for columns constant on the fit rows.
 *   mu_sd  device float[n_feat][2] out */
int kaldo_standardize(int64_t n, int32_t n_feat, float* X, int64_t n_fit, float* mu_sd,
                      void* stream);

/* kaldo_surrogate_targets -- y_k = (ln gamma[modes[k]] - mu) / sd (float32)
 * with mu, sd the mean and population std of ln gamma over the listed modes.
 *   gamma    device double[N_q*nb3] rad/ps, > 0 at the listed modes
 *   y        device float[n]; y_mu_sd device float[2] out */
int kaldo_surrogate_targets(const double* gamma, const int32_t* modes, int64_t n, float* y,
                            float* y_mu_sd, void* stream);

/* Parameters per ensemble member for n_in inputs (-1 if n_in not in 1..32):
 * W0 [n_in][64], b0 [64], W1..W3 [64][64] each followed by its bias [64],
 * head W4 [64], b4 [1]; row-major, in that order. */
int32_t kaldo_mlp_param_count(int32_t n_in);

/* Device workspace bytes kaldo_mlp_train needs. */
size_t kaldo_mlp_workspace(int32_t n_in, int32_t n_members, int32_t n_samples);

/* kaldo_mlp_train -- full-batch training of an ensemble of n_members MLPs
 * (4 hidden layers of 64 tanh units, linear head), FP32.  Member e minimises
 *   L_e = sum_i c_ei (f_e(x_i) - y_i)^2 / sum_i c_ei
 * (c = bootstrap counts) with `steps` Adam steps (b1 0.9, b2 0.999, eps 1e-8,
 * bias-corrected, learning rate lr).  Gradients are reduced in a fixed order:
 * identical inputs give identical parameters.
 *   X        device float[n_samples][n_in] (n_in <= 32)
 *   y        device float[n_samples]
 *   counts   device float[n_members][n_samples] (integers >= 0, sum > 0)
 *   params   device float[n_members][P] in: initial, out: trained
 *   losses   device float[n_members][steps] or NULL: L_e before each step
 *   grad_out device float[n_members][P] or NULL: gradient of the last step
 * One cooperative launch whose workgroups meet at a grid barrier twice per
 * step.  Returns EUNSUPPORTED when the grid cannot be co-resident.  This
 * call synchronises `stream` and returns EDEVICE if a barrier timed out. */
int kaldo_mlp_train(int32_t n_in, int32_t n_members, int32_t n_samples, const float* X,
                    const float* y, const float* counts, float* params, int32_t steps, float lr,
                    void* workspace, size_t workspace_bytes, float* losses, float* grad_out,
                    void* stream);

/* kaldo_mlp_predict -- ensemble forward pass: per row the mean and the
 * population std over members of the outputs (n_members <= 16).
 *   X       device float[n][n_in]; params device float[n_members][P]
 *   mean, spread  device float[n] out */
int kaldo_mlp_predict(int32_t n_in, int32_t n_members, int64_t n, const float* X,
                      const float* params, float* mean, float* spread, void* stream);

/* kaldo_surrogate_domain -- per feature column the [min, max] over the first
 * n_fit rows of X (device float[n][n_feat], n_feat <= 32); inside[k]
 * (device uint8[n]) = 1 when every feature of row k lies in those ranges.
 * Rows outside the training domain are extrapolations: the gate sends them
 * to the exact path whatever the ensemble's spread. */
int kaldo_surrogate_domain(int64_t n, int32_t n_feat, const float* X, int64_t n_fit,
                           uint8_t* inside, void* stream);

/* kaldo_gate_score -- per row the first-order conductivity error the
 * ensemble's disagreement implies:
 *   score[k] = w / G_pred * spread[k] * sd,   G_pred = exp(mean[k] sd + mu),
 *   w = star_size[q] c(omega)/k_B |v|^2 (Eq. heatcap; trace of Eq. rta's
 *   summand without the constant factor),
 * with (mu, sd) = y_mu_sd; +inf where inside is given and inside[k] == 0.
 *   modes device int32[n]; mean, spread device float[n]; score device float[n] */
int kaldo_gate_score(int64_t n, const int32_t* modes, const float* mean, const float* spread,
                     const float* y_mu_sd, const double* omega, const double* vel,
                     const int32_t* star_size, int32_t nb3, double temperature,
                     const uint8_t* inside, float* score, void* stream);

/* kaldo_gate_calibrate -- gate threshold from n held-out rows (n <= 4096).
 * Row k (mode modes[k]): w as in kaldo_gate_score, predicted Gamma =
 * exp(mean[k] sd + mu).  Rows are taken in ascending score, equal scores as
 * one group; a group is accepted while
 *   |sum_accepted w (1/G_pred - 1/G_true)| <= tol sum_all w / G_true.
 * *tau (device float) = the next float above the last accepted score, 0 if
 * none: rows with score < tau use the network. */
int kaldo_gate_calibrate(int64_t n, const int32_t* modes, const double* gamma, const float* mean,
                         const float* y_mu_sd, const float* score, const double* omega,
                         const double* vel, const int32_t* star_size, int32_t nb3,
                         double temperature, double tol, float* tau, void* stream);

/* kaldo_gate_select -- rows k with score[k] >= *tau whose mode is not yet
 * computed (computed[modes[k]] == 0) are appended in row order to fallback
 * (device int32[n]) and marked computed; *n_fallback (device int32) = their
 * count.  The listed modes must be distinct; computed is device
 * uint8[n_modes] and rows whose mode lies outside [0, n_modes) are skipped. */
int kaldo_gate_select(int64_t n, int64_t n_modes, const int32_t* modes, const float* score,
                      const float* tau, uint8_t* computed, int32_t* fallback, int32_t* n_fallback,
                      void* stream);

/* kaldo_surrogate_fill -- gamma[modes[k]] = exp(mean[k] sd + mu) for rows whose
 * mode is not computed; other entries untouched.  computed is device
 * uint8[n_modes], gamma device double[n_modes]; rows whose mode lies outside
 * [0, n_modes) are skipped. */
int kaldo_surrogate_fill(int64_t n, int64_t n_modes, const int32_t* modes, const float* mean,
                         const float* y_mu_sd, const uint8_t* computed, double* gamma,
                         void* stream);

/* kaldo_star_map -- full-grid linewidths from the representatives':
 * gamma[q][s] = mean of gamma_ir[rep(q)][s'] over the frequency cluster
 * (|d nu| < 1e-4 THz) of s at rep(q).  Linewidths are invariant under the
 * crystal's point operations; cluster averaging removes the gauge freedom
 * of degenerate modes.  gamma must not alias gamma_ir. */
int kaldo_star_map(const int32_t* mesh, int32_t nb3, const int32_t* ir_of_q,
                   const double* omega, const double* gamma_ir, double* gamma, void* stream);

/* Per-kernel timing.  kaldo_profile_begin() makes every later kernel launch
 * of the library record a HIP event before and after it on its launch
 * stream; kaldo_profile_end() waits for those events, writes up to
 * `capacity` records (one per kernel name, in first-launch order) and sets
 * *n_out to the number of distinct kernels, then switches timing off.
 * Process-wide; calls from several threads are serialised. */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
} kaldo_kernel_time;
int kaldo_profile_begin(void);
int kaldo_profile_end(kaldo_kernel_time* out, int32_t capacity, int32_t* n_out);

/* Thread-local message for the last failing call in this thread. */
const char* kaldo_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int kaldo_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KALDO_H */
