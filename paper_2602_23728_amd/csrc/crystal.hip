// Crystal handle: validation, host-side index planning of the FC3 COO, and
// upload of every table the kernels read.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <numeric>
#include <tuple>

#include "common.h"

namespace kaldo {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

void reciprocal(const double* a, double* b) {
  // b_c = 2 pi (a_{c+1} x a_{c+2}) / (a_0 . (a_1 x a_2))
  auto cross = [](const double* u, const double* v, double* w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  double c[3];
  cross(a + 3, a + 6, c);
  double vol = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
  for (int r = 0; r < 3; ++r) {
    double w[3];
    cross(a + 3 * ((r + 1) % 3), a + 3 * ((r + 2) % 3), w);
    for (int k = 0; k < 3; ++k) b[3 * r + k] = kTwoPi * w[k] / vol;
  }
}

template <typename T>
static int upload(kaldo_crystal* c, T** dst, const std::vector<T>& src) {
  size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    set_error("hipMalloc failed for " + std::to_string(bytes) + " bytes");
    return KALDO_ENOMEM;
  }
  c->allocations.push_back(p);
  if (!src.empty()) KALDO_HIP(hipMemcpy(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  *dst = static_cast<T*>(p);
  return KALDO_OK;
}

static void free_all(kaldo_crystal* c) {
  for (void* p : c->allocations) (void)hipFree(p);
  c->allocations.clear();
}

// Phi3 symmetric in its last two slots: every (i, j, k) carries the value of
// (i, k, j) (duplicate COO entries summed) to within 1e-12 of the largest
// |value|.  A derivative tensor is, so the linewidth kernels may then visit
// each mirrored partner pair once.
static bool fc3_symmetric_jk(int64_t nnz, const int32_t* fi, const int32_t* fj, const int32_t* fk,
                             const double* fv) {
  std::map<std::array<int32_t, 3>, double> m;
  for (int64_t t = 0; t < nnz; ++t) m[{fi[t], fj[t], fk[t]}] += fv[t];
  double vmax = 0.0;
  for (const auto& kv : m) vmax = std::max(vmax, std::fabs(kv.second));
  const double tol = 1e-12 * vmax;
  for (const auto& kv : m) {
    const auto it = m.find({kv.first[0], kv.first[2], kv.first[1]});
    const double v2 = it == m.end() ? 0.0 : it->second;
    if (std::fabs(kv.second - v2) > tol) return false;
  }
  return true;
}

static int build_bloch(kaldo_crystal* c, int64_t nnz, const int32_t* fi, const int32_t* fj,
                       const int32_t* fk, const double* fv) {
  const int nb = c->nb;
  struct Contrib { int32_t i, l2; double coef; int64_t order; };
  // key: (d0, d1, d2, jc, kc)
  std::map<std::array<int32_t, 5>, std::vector<Contrib>> groups;
  for (int64_t t = 0; t < nnz; ++t) {
    int32_t jr = (fj[t] / 3) / nb, jb = (fj[t] / 3) % nb, kr = (fk[t] / 3) / nb,
            kb = (fk[t] / 3) % nb, ib = fi[t] / 3;
    std::array<int32_t, 5> key = {c->rep[3 * jr] - c->rep[3 * kr],
                                  c->rep[3 * jr + 1] - c->rep[3 * kr + 1],
                                  c->rep[3 * jr + 2] - c->rep[3 * kr + 2],
                                  jb * 3 + fj[t] % 3, kb * 3 + fk[t] % 3};
    double coef = fv[t] / std::sqrt(c->mass[ib] * c->mass[jb] * c->mass[kb]);
    groups[key].push_back({fi[t], kr, coef, t});
  }
  std::vector<int32_t> dvec, d_ptr, e_jc, e_kc, t_ptr, t_i, t_l2;
  std::vector<double> t_coef;
  std::array<int32_t, 3> cur = {INT32_MIN, INT32_MIN, INT32_MIN};
  t_ptr.push_back(0);
  for (auto& kv : groups) {
    const auto& key = kv.first;
    std::array<int32_t, 3> d = {key[0], key[1], key[2]};
    if (d != cur) {
      cur = d;
      dvec.insert(dvec.end(), d.begin(), d.end());
      d_ptr.push_back(static_cast<int32_t>(e_jc.size()));
    }
    e_jc.push_back(key[3]);
    e_kc.push_back(key[4]);
    auto v = kv.second;
    std::sort(v.begin(), v.end(), [](const Contrib& a, const Contrib& b) {
      return std::tie(a.i, a.l2, a.order) < std::tie(b.i, b.l2, b.order);
    });
    for (auto& x : v) {
      t_i.push_back(x.i);
      t_l2.push_back(x.l2);
      t_coef.push_back(x.coef);
    }
    t_ptr.push_back(static_cast<int32_t>(t_i.size()));
  }
  d_ptr.push_back(static_cast<int32_t>(e_jc.size()));
  // atom blocks (jb, kb, d), sorted by (jb, kb, d)
  const int n_d = static_cast<int>(dvec.size() / 3);
  std::map<std::array<int32_t, 3>, int32_t> blocks;
  for (int d = 0; d < n_d; ++d)
    for (int e = d_ptr[d]; e < d_ptr[d + 1]; ++e) blocks[{e_jc[e] / 3, e_kc[e] / 3, d}] = 0;
  std::vector<int32_t> blk_d, pair_ptr(nb * nb + 1, 0), e_blk(e_jc.size()), e_bg(e_jc.size());
  int32_t nblk = 0;
  for (auto& kv : blocks) {
    kv.second = nblk++;
    blk_d.push_back(kv.first[2]);
    pair_ptr[kv.first[0] * nb + kv.first[1] + 1]++;
  }
  for (int k = 0; k < nb * nb; ++k) pair_ptr[k + 1] += pair_ptr[k];
  for (int d = 0; d < n_d; ++d)
    for (int e = d_ptr[d]; e < d_ptr[d + 1]; ++e) {
      e_blk[e] = blocks[{e_jc[e] / 3, e_kc[e] / 3, d}];
      e_bg[e] = (e_jc[e] % 3) * 3 + e_kc[e] % 3;
    }
  // balanced work list for the 16x16 B_s tiles of the MFMA kernel
  std::vector<int4> bwork(256, int4{-1, 0, 0, 0});
  if (3 * nb <= 16) {
    struct W { int pos, lo, hi, bg; };
    std::vector<W> ws;
    for (int jc = 0; jc < 3 * nb; ++jc)
      for (int kc = 0; kc < 3 * nb; ++kc) {
        const int pr = (jc / 3) * nb + kc / 3;
        ws.push_back({jc * 17 + kc, pair_ptr[pr], pair_ptr[pr + 1], (jc % 3) * 3 + kc % 3});
      }
    std::stable_sort(ws.begin(), ws.end(),
                     [](const W& a, const W& b) { return a.hi - a.lo > b.hi - b.lo; });
    for (size_t e = 0; e < ws.size(); ++e) {
      // serpentine deal over the 64 lanes keeps per-lane block counts even
      const int slot = static_cast<int>(e / 64), l = static_cast<int>(e % 64);
      const int lane = (slot & 1) ? 63 - l : l;
      bwork[slot * 64 + lane] = int4{ws[e].pos, ws[e].lo, ws[e].hi, ws[e].bg};
    }
  }
  Fc3Bloch& b = c->bloch;
  b.n_blk = nblk;
  b.sym_jk = fc3_symmetric_jk(nnz, fi, fj, fk, fv) ? 1 : 0;
  b.n_d = static_cast<int>(dvec.size() / 3);
  b.n_e = static_cast<int>(e_jc.size());
  b.n_t = static_cast<int>(t_i.size());
  int rc;
  if ((rc = upload(c, &b.dvec, dvec))) return rc;
  if ((rc = upload(c, &b.d_ptr, d_ptr))) return rc;
  if ((rc = upload(c, &b.e_jc, e_jc))) return rc;
  if ((rc = upload(c, &b.e_kc, e_kc))) return rc;
  if ((rc = upload(c, &b.t_ptr, t_ptr))) return rc;
  if ((rc = upload(c, &b.t_i, t_i))) return rc;
  if ((rc = upload(c, &b.t_l2, t_l2))) return rc;
  if ((rc = upload(c, &b.t_coef, t_coef))) return rc;
  if ((rc = upload(c, &b.e_blk, e_blk))) return rc;
  if ((rc = upload(c, &b.e_bg, e_bg))) return rc;
  if ((rc = upload(c, &b.blk_d, blk_d))) return rc;
  if ((rc = upload(c, &b.pair_ptr, pair_ptr))) return rc;
  if ((rc = upload(c, &b.bwork, bwork))) return rc;
  return KALDO_OK;
}

static int build_gamma(kaldo_crystal* c, int64_t nnz, const int32_t* fi, const int32_t* fj,
                       const int32_t* fk, const double* fv) {
  const int nb3 = c->nb3;
  std::vector<int64_t> idx(nnz);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return std::make_tuple(fj[a], fk[a], fi[a], a) < std::make_tuple(fj[b], fk[b], fi[b], b);
  });
  std::vector<int32_t> row_ptr(nb3 + 1, 0), col, t_ptr, t_a;
  std::vector<double> t_coef;
  t_ptr.push_back(0);
  int32_t pb = -1, pc = -1;
  for (int64_t n = 0; n < nnz; ++n) {
    int64_t t = idx[n];
    int32_t b = fj[t], cc = fk[t];
    if (b != pb || cc != pc) {
      if (pb >= 0) t_ptr.push_back(static_cast<int32_t>(t_a.size()));
      col.push_back(cc);
      row_ptr[b + 1]++;
      pb = b;
      pc = cc;
    }
    int32_t a = fi[t];
    t_a.push_back(a);
    t_coef.push_back(fv[t] / std::sqrt(c->mass[a / 3] * c->mass[b / 3] * c->mass[cc / 3]));
  }
  if (pb >= 0) t_ptr.push_back(static_cast<int32_t>(t_a.size()));
  for (int r = 0; r < nb3; ++r) row_ptr[r + 1] += row_ptr[r];
  const int n_rt = (nb3 + kSpmmRows - 1) / kSpmmRows;
  std::vector<int32_t> tile_u_ptr(1, 0), tile_u, col_local(col.size());
  int max_u = 0, g_max_entries = 0;
  for (int t = 0; t < n_rt; ++t) {
    const int r0 = t * kSpmmRows, r1 = std::min(nb3, r0 + kSpmmRows);
    std::vector<int32_t> u(col.begin() + row_ptr[r0], col.begin() + row_ptr[r1]);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    for (int k = row_ptr[r0]; k < row_ptr[r1]; ++k)
      col_local[k] = static_cast<int32_t>(std::lower_bound(u.begin(), u.end(), col[k]) - u.begin());
    tile_u.insert(tile_u.end(), u.begin(), u.end());
    tile_u_ptr.push_back(static_cast<int32_t>(tile_u.size()));
    max_u = std::max<int>(max_u, static_cast<int>(u.size()));
    g_max_entries = std::max(g_max_entries, row_ptr[r1] - row_ptr[r0]);
  }
  int max_row = 0;
  for (int r = 0; r < nb3; ++r) max_row = std::max(max_row, row_ptr[r + 1] - row_ptr[r]);
  std::vector<int32_t> col_ell((size_t)max_row * nb3, 0);
  for (int r = 0; r < nb3; ++r)
    for (int k = row_ptr[r]; k < row_ptr[r + 1]; ++k) col_ell[(size_t)(k - row_ptr[r]) * nb3 + r] = col_local[k];
  Fc3Gamma& g = c->gamma;
  g.max_row = max_row;
  g.n_rtiles = n_rt;
  g.max_u = max_u;
  g.max_tile_entries = g_max_entries;
  g.n_bc = static_cast<int>(col.size());
  g.n_t = static_cast<int>(t_a.size());
  int rc;
  if ((rc = upload(c, &g.row_ptr, row_ptr))) return rc;
  if ((rc = upload(c, &g.col, col))) return rc;
  if ((rc = upload(c, &g.t_ptr, t_ptr))) return rc;
  if ((rc = upload(c, &g.t_a, t_a))) return rc;
  if ((rc = upload(c, &g.t_coef, t_coef))) return rc;
  if ((rc = upload(c, &g.tile_u_ptr, tile_u_ptr))) return rc;
  if ((rc = upload(c, &g.tile_u, tile_u))) return rc;
  if ((rc = upload(c, &g.col_ell, col_ell))) return rc;
  return KALDO_OK;
}

}  // namespace kaldo

using namespace kaldo;

extern "C" const char* kaldo_last_error(void) { return g_last_error.c_str(); }

extern "C" int kaldo_version(void) { return 100; }

extern "C" int kaldo_crystal_create(int32_t n_basis, const double* lattice, const double* mass,
                                    int32_t n_rep, const int32_t* rep, const double* fc2,
                                    int64_t nnz, const int32_t* fc3_i, const int32_t* fc3_j,
                                    const int32_t* fc3_k, const double* fc3_val,
                                    kaldo_crystal** out) {
  KALDO_REQUIRE(out != nullptr, "kaldo_crystal_create: out is NULL");
  *out = nullptr;
  KALDO_REQUIRE(n_basis >= 1 && n_rep >= 1 && nnz >= 0, "kaldo_crystal_create: bad sizes");
  KALDO_REQUIRE(lattice && mass && rep && fc2, "kaldo_crystal_create: NULL array");
  KALDO_REQUIRE(nnz == 0 || (fc3_i && fc3_j && fc3_k && fc3_val),
                "kaldo_crystal_create: NULL FC3 array");
  KALDO_REQUIRE(rep[0] == 0 && rep[1] == 0 && rep[2] == 0,
                "kaldo_crystal_create: rep[0] must be (0,0,0)");
  const int nb3 = 3 * n_basis;
  double vol = lattice[0] * (lattice[4] * lattice[8] - lattice[5] * lattice[7]) -
               lattice[1] * (lattice[3] * lattice[8] - lattice[5] * lattice[6]) +
               lattice[2] * (lattice[3] * lattice[7] - lattice[4] * lattice[6]);
  KALDO_REQUIRE(std::isfinite(vol) && std::fabs(vol) > 1e-12,
                "kaldo_crystal_create: singular lattice");
  for (int i = 0; i < n_basis; ++i)
    KALDO_REQUIRE(std::isfinite(mass[i]) && mass[i] > 0, "kaldo_crystal_create: mass <= 0");
  const size_t n2 = static_cast<size_t>(nb3) * n_rep * nb3;
  for (size_t k = 0; k < n2; ++k)
    KALDO_REQUIRE(std::isfinite(fc2[k]), "kaldo_crystal_create: non-finite FC2");
  const int32_t jmax = 3 * n_basis * n_rep;
  for (int64_t t = 0; t < nnz; ++t) {
    KALDO_REQUIRE(fc3_i[t] >= 0 && fc3_i[t] < nb3, "kaldo_crystal_create: fc3_i out of range");
    KALDO_REQUIRE(fc3_j[t] >= 0 && fc3_j[t] < jmax, "kaldo_crystal_create: fc3_j out of range");
    KALDO_REQUIRE(fc3_k[t] >= 0 && fc3_k[t] < jmax, "kaldo_crystal_create: fc3_k out of range");
    KALDO_REQUIRE(std::isfinite(fc3_val[t]), "kaldo_crystal_create: non-finite FC3 value");
  }
  auto* c = new (std::nothrow) kaldo_crystal_s();
  if (!c) {
    set_error("kaldo_crystal_create: host allocation failed");
    return KALDO_ENOMEM;
  }
  c->nb = n_basis;
  c->nb3 = nb3;
  c->n_rep = n_rep;
  std::copy(lattice, lattice + 9, c->lattice);
  c->volume = std::fabs(vol);
  c->mass.assign(mass, mass + n_basis);
  c->rep.assign(rep, rep + 3 * n_rep);
  c->fc2.assign(fc2, fc2 + n2);
  std::vector<double> scaled(n2), repcart(3 * n_rep);
  for (int a = 0; a < nb3; ++a)
    for (int l = 0; l < n_rep; ++l)
      for (int b = 0; b < nb3; ++b) {
        size_t k = (static_cast<size_t>(a) * n_rep + l) * nb3 + b;
        scaled[k] = fc2[k] / std::sqrt(mass[a / 3] * mass[b / 3]);
      }
  for (int l = 0; l < n_rep; ++l)
    for (int x = 0; x < 3; ++x)
      repcart[3 * l + x] = rep[3 * l] * lattice[x] + rep[3 * l + 1] * lattice[3 + x] +
                           rep[3 * l + 2] * lattice[6 + x];
  int rc = upload(c, &c->d_fc2, scaled);
  if (!rc) rc = upload(c, &c->d_rep, c->rep);
  if (!rc) rc = upload(c, &c->d_repcart, repcart);
  if (!rc) rc = upload(c, &c->d_flags, std::vector<int32_t>(1, 0));
  if (!rc) rc = build_bloch(c, nnz, fc3_i, fc3_j, fc3_k, fc3_val);
  if (!rc && n_rep == 1) rc = build_gamma(c, nnz, fc3_i, fc3_j, fc3_k, fc3_val);
  if (rc) {
    free_all(c);
    delete c;
    return rc;
  }
  *out = c;
  return KALDO_OK;
}

extern "C" int kaldo_device_status(kaldo_crystal* c, void* stream) {
  KALDO_REQUIRE(c != nullptr, "kaldo_device_status: NULL handle");
  KALDO_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  int32_t flags = 0;
  KALDO_HIP(hipMemcpy(&flags, c->d_flags, sizeof(flags), hipMemcpyDeviceToHost));
  if (flags == 0) return KALDO_OK;
  const int32_t zero = 0;
  KALDO_HIP(hipMemcpy(c->d_flags, &zero, sizeof(zero), hipMemcpyHostToDevice));
  std::string msg = "kaldo_device_status:";
  if (flags & kFlagNonFinite) msg += " non-finite value in a device input (omega, eta, v or Gamma);";
  if (flags & kFlagSubset) msg += " modes_subset index out of range;";
  if (flags & kFlagCache) msg += " temperature-cache row or pair index out of range;";
  if (flags & kFlagImaginary) msg += " imaginary mode (omega^2 < 0) above nu_min;";
  if (flags & kFlagNoConverge) msg += " eigen-solver did not converge within its sweep cap;";
  if (flags & kFlagSingular) msg += " zero pivot in the LU factorisation of the scattering matrix;";
  set_error(msg);
  return (flags & (kFlagNonFinite | kFlagSubset | kFlagCache)) ? KALDO_EINVAL : KALDO_ENUMERIC;
}

extern "C" int kaldo_crystal_destroy(kaldo_crystal* c) {
  if (!c) return KALDO_OK;
  free_all(c);
  delete c;
  return KALDO_OK;
}
