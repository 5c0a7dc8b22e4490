// Native generator of the explicit pressure-correction workload (Sec. 5.3): graded
// tensor grids, Q1 velocity on the refined grid and Q1 pressure on the coarse one, and
// every matrix of the time step as sums of Kronecker products of one-dimensional P1
// matrices (exact for Q1 on boxes).  Host C++17.
#include "../../../include/mgns.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

struct Fail : std::runtime_error {
  int code;
  Fail(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- one dimension
// tridiagonal matrix: v[i] = entries (i, i-1), (i, i), (i, i+1)
using Tri = std::vector<std::array<double, 3>>;

struct P1 {
  Tri M, K, C;            // mass, stiffness, C_ij = (phi_j, phi_i')
  std::vector<double> m;  // lumped mass = integral of phi_i
};

P1 p1_matrices(const std::vector<double>& x) {
  const size_t n = x.size();
  P1 o;
  o.M.assign(n, {0.0, 0.0, 0.0});
  o.K.assign(n, {0.0, 0.0, 0.0});
  o.C.assign(n, {0.0, 0.0, 0.0});
  o.m.assign(n, 0.0);
  for (size_t e = 0; e + 1 < n; ++e) {
    const double h = x[e + 1] - x[e];
    const double m6 = h / 6.0, k1 = 1.0 / h;
    o.M[e][1] += m6 * 2.0;
    o.M[e][2] += m6;
    o.M[e + 1][0] += m6;
    o.M[e + 1][1] += m6 * 2.0;
    o.K[e][1] += k1;
    o.K[e][2] += -k1;
    o.K[e + 1][0] += -k1;
    o.K[e + 1][1] += k1;
    // phi_e' = -1/h, phi_{e+1}' = 1/h on the cell, and the integral of each hat is h/2
    o.C[e][1] += -0.5;
    o.C[e][2] += -0.5;
    o.C[e + 1][0] += 0.5;
    o.C[e + 1][1] += 0.5;
    o.m[e] += h / 2;
    o.m[e + 1] += h / 2;
  }
  return o;
}

// sparse row of a one-dimensional rectangular matrix: (column, value) ascending
using Row1 = std::vector<std::pair<int32_t, double>>;

// nodal interpolation of the coarse hats at the fine nodes (fine x coarse)
std::vector<Row1> interp_1d(const std::vector<double>& xc, const std::vector<double>& xf) {
  std::vector<Row1> P(xf.size());
  const int32_t nc = int32_t(xc.size());
  for (size_t i = 0; i < xf.size(); ++i) {
    const double x = xf[i];
    int32_t e = int32_t(std::upper_bound(xc.begin(), xc.end(), x) - xc.begin()) - 1;
    e = std::min(std::max(e, 0), nc - 2);
    const double t = (x - xc[size_t(e)]) / (xc[size_t(e) + 1] - xc[size_t(e)]);
    if (1.0 - t != 0.0) P[i].push_back({e, 1.0 - t});
    if (t != 0.0) P[i].push_back({e + 1, t});
  }
  return P;
}

// (A P) for tridiagonal A (fine x fine) and P (fine x coarse)
std::vector<Row1> tri_times(const Tri& A, const std::vector<Row1>& P) {
  const int64_t n = int64_t(A.size());
  std::vector<Row1> out(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) {
    std::map<int32_t, double> acc;
    for (int d = 0; d < 3; ++d) {
      const int64_t j = i + d - 1;
      if (j < 0 || j >= n) continue;
      for (const auto& [q, w] : P[size_t(j)]) acc[q] += A[size_t(i)][size_t(d)] * w;
    }
    for (const auto& [q, v] : acc) out[size_t(i)].push_back({q, v});
  }
  return out;
}

// union of the column sets of two rows, with both rows' values (0 where absent)
struct Row2 {
  std::vector<int32_t> col;
  std::vector<double> a, b;
};
std::vector<Row2> merge_rows(const std::vector<Row1>& A, const std::vector<Row1>& B) {
  std::vector<Row2> out(A.size());
  for (size_t i = 0; i < A.size(); ++i) {
    std::map<int32_t, std::pair<double, double>> m;
    for (const auto& [q, v] : A[i]) m[q].first = v;
    for (const auto& [q, v] : B[i]) m[q].second = v;
    for (const auto& [q, v] : m) {
      out[i].col.push_back(q);
      out[i].a.push_back(v.first);
      out[i].b.push_back(v.second);
    }
  }
  return out;
}

std::vector<double> graded(int32_t n, int axis, double length) {
  std::vector<double> c(size_t(n) + 1);
  for (int32_t i = 0; i <= n; ++i) {
    const double t = double(i);
    c[size_t(i)] = axis < 2 ? 0.5 * (1.0 - std::cos(t * kPi / n)) : 1.0 + std::sin((t - n) * kPi / (2.0 * n));
  }
  c.front() = 0.0;
  c.back() = 1.0;
  for (double& v : c) v *= length;
  return c;
}

std::vector<double> refine(const std::vector<double>& c) {
  std::vector<double> o(2 * c.size() - 1);
  for (size_t i = 0; i < c.size(); ++i) o[2 * i] = c[i];
  for (size_t i = 0; i + 1 < c.size(); ++i) o[2 * i + 1] = 0.5 * (c[i] + c[i + 1]);
  return o;
}

std::vector<double> every_other(const std::vector<double>& c) {
  std::vector<double> o;
  for (size_t i = 0; i < c.size(); i += 2) o.push_back(c[i]);
  return o;
}

// ---------------------------------------------------------------- three dimensions
struct Csr {
  std::vector<int32_t> rowptr, col;
};

struct PLevel {
  int32_t n = 0;
  Csr A;
  std::vector<double> a;
  Csr P;
  std::vector<double> p;
  int32_t p_cols = 0;
  std::vector<uint8_t> mask;
};

// pressure Laplacian on the tensor grid with node 0 pinned (identity row and column)
void pressure_operator(const std::array<std::vector<double>, 3>& x, PLevel& L) {
  const P1 X = p1_matrices(x[0]), Y = p1_matrices(x[1]), Z = p1_matrices(x[2]);
  const int32_t nx = int32_t(x[0].size()), ny = int32_t(x[1].size()), nz = int32_t(x[2].size());
  L.n = nx * ny * nz;
  L.A.rowptr.assign(1, 0);
  for (int32_t k = 0; k < nz; ++k)
    for (int32_t j = 0; j < ny; ++j)
      for (int32_t i = 0; i < nx; ++i) {
        const int32_t row = (k * ny + j) * nx + i;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int32_t kk = k + dz, jj = j + dy, ii = i + dx;
              if (kk < 0 || kk >= nz || jj < 0 || jj >= ny || ii < 0 || ii >= nx) continue;
              const int32_t col = (kk * ny + jj) * nx + ii;
              if ((row == 0 || col == 0) && row != col) continue;
              double v;
              if (row == 0) {
                v = 1.0;
              } else {
                const double mx = X.M[size_t(i)][size_t(dx + 1)], kx = X.K[size_t(i)][size_t(dx + 1)];
                const double my = Y.M[size_t(j)][size_t(dy + 1)], ky = Y.K[size_t(j)][size_t(dy + 1)];
                const double mz = Z.M[size_t(k)][size_t(dz + 1)], kz = Z.K[size_t(k)][size_t(dz + 1)];
                v = mz * (my * kx) + mz * (ky * mx) + kz * (my * mx);
              }
              L.A.col.push_back(col);
              L.a.push_back(v);
            }
        L.A.rowptr.push_back(int32_t(L.A.col.size()));
      }
  L.mask.assign(size_t(L.n), 0);
  L.mask[0] = 1;
}

// scalar prolongation fine x coarse: tensor product of the 1D nodal interpolations
void pressure_prolongation(const std::array<std::vector<double>, 3>& xc, const std::array<std::vector<double>, 3>& xf,
                           PLevel& L) {
  const auto Px = interp_1d(xc[0], xf[0]), Py = interp_1d(xc[1], xf[1]), Pz = interp_1d(xc[2], xf[2]);
  const int32_t ncx = int32_t(xc[0].size()), ncy = int32_t(xc[1].size());
  L.p_cols = ncx * ncy * int32_t(xc[2].size());
  L.P.rowptr.assign(1, 0);
  for (size_t k = 0; k < xf[2].size(); ++k)
    for (size_t j = 0; j < xf[1].size(); ++j)
      for (size_t i = 0; i < xf[0].size(); ++i) {
        for (const auto& [qz, wz] : Pz[k])
          for (const auto& [qy, wy] : Py[j])
            for (const auto& [qx, wx] : Px[i]) {
              L.P.col.push_back((qz * ncy + qy) * ncx + qx);
              L.p.push_back(wz * (wy * wx));
            }
        L.P.rowptr.push_back(int32_t(L.P.col.size()));
      }
}

}  // namespace

struct mgns_problem {
  mgns_config cfg{};
  int32_t n_v = 0, n_p = 0;
  Csr V;
  std::vector<double> K, C[3];
  Csr G;
  std::vector<double> Gv[3];
  Csr D;
  std::vector<double> Dv[3];
  std::vector<double> m_v, m_p, dir_val, coords;
  std::vector<uint8_t> dir_mask;
  std::vector<PLevel> levels;    // coarsest first
};

namespace {

void build(mgns_problem& P) {
  const mgns_config& c = P.cfg;
  std::array<std::vector<double>, 3> xp, xv;
  for (int a = 0; a < 3; ++a) {
    xp[size_t(a)] = graded(c.cells[a], a, c.length[a]);
    xv[size_t(a)] = refine(xp[size_t(a)]);
  }
  const P1 X = p1_matrices(xv[0]), Y = p1_matrices(xv[1]), Z = p1_matrices(xv[2]);
  const int32_t nx = int32_t(xv[0].size()), ny = int32_t(xv[1].size()), nz = int32_t(xv[2].size());
  P.n_v = nx * ny * nz;
  // velocity matrices on the 27-point pattern, lumped mass, boundary data, coordinates
  P.V.rowptr.assign(1, 0);
  P.m_v.resize(size_t(P.n_v));
  P.dir_mask.assign(size_t(P.n_v) * 3, 0);
  P.dir_val.assign(size_t(P.n_v) * 3, 0.0);
  P.coords.resize(size_t(P.n_v) * 3);
  for (int32_t k = 0; k < nz; ++k)
    for (int32_t j = 0; j < ny; ++j)
      for (int32_t i = 0; i < nx; ++i) {
        const int64_t row = (int64_t(k) * ny + j) * nx + i;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int32_t kk = k + dz, jj = j + dy, ii = i + dx;
              if (kk < 0 || kk >= nz || jj < 0 || jj >= ny || ii < 0 || ii >= nx) continue;
              const double mx = X.M[size_t(i)][size_t(dx + 1)], kx = X.K[size_t(i)][size_t(dx + 1)],
                           cx = X.C[size_t(i)][size_t(dx + 1)];
              const double my = Y.M[size_t(j)][size_t(dy + 1)], ky = Y.K[size_t(j)][size_t(dy + 1)],
                           cy = Y.C[size_t(j)][size_t(dy + 1)];
              const double mz = Z.M[size_t(k)][size_t(dz + 1)], kz = Z.K[size_t(k)][size_t(dz + 1)],
                           cz = Z.C[size_t(k)][size_t(dz + 1)];
              P.V.col.push_back((kk * ny + jj) * nx + ii);
              P.K.push_back(mz * (my * kx) + mz * (ky * mx) + kz * (my * mx));
              P.C[0].push_back(mz * (my * cx));
              P.C[1].push_back(mz * (cy * mx));
              P.C[2].push_back(cz * (my * mx));
            }
        P.V.rowptr.push_back(int32_t(P.V.col.size()));
        P.m_v[size_t(row)] = Z.m[size_t(k)] * (Y.m[size_t(j)] * X.m[size_t(i)]);
        const bool bnd = i == 0 || i == nx - 1 || j == 0 || j == ny - 1 || k == 0 || k == nz - 1;
        for (int cc = 0; cc < 3; ++cc) P.dir_mask[size_t(row) * 3 + cc] = bnd ? 1 : 0;
        if (i == nx - 1) P.dir_val[size_t(row) * 3 + 1] = 1.0;   // moving wall x = L0: u = (0, 1, 0)
        P.coords[size_t(row) * 3 + 0] = xv[0][size_t(i)];
        P.coords[size_t(row) * 3 + 1] = xv[1][size_t(j)];
        P.coords[size_t(row) * 3 + 2] = xv[2][size_t(k)];
      }
  // coupling G_a = C_a P = (M_z P_z) (x) (M_y P_y) (x) (C_x P_x) etc.
  std::array<std::vector<Row2>, 3> R;   // per axis: (M P, C P) on the union pattern
  const P1* F[3] = {&X, &Y, &Z};
  for (int a = 0; a < 3; ++a) {
    const auto Pa = interp_1d(xp[size_t(a)], xv[size_t(a)]);
    R[size_t(a)] = merge_rows(tri_times(F[a]->M, Pa), tri_times(F[a]->C, Pa));
  }
  const int32_t npx = int32_t(xp[0].size()), npy = int32_t(xp[1].size()), npz = int32_t(xp[2].size());
  P.n_p = npx * npy * npz;
  P.G.rowptr.assign(1, 0);
  for (int32_t k = 0; k < nz; ++k)
    for (int32_t j = 0; j < ny; ++j)
      for (int32_t i = 0; i < nx; ++i) {
        const Row2 &rz = R[2][size_t(k)], &ry = R[1][size_t(j)], &rx = R[0][size_t(i)];
        for (size_t a = 0; a < rz.col.size(); ++a)
          for (size_t b = 0; b < ry.col.size(); ++b)
            for (size_t d = 0; d < rx.col.size(); ++d) {
              P.G.col.push_back((rz.col[a] * npy + ry.col[b]) * npx + rx.col[d]);
              P.Gv[0].push_back(rz.a[a] * (ry.a[b] * rx.b[d]));
              P.Gv[1].push_back(rz.a[a] * (ry.b[b] * rx.a[d]));
              P.Gv[2].push_back(rz.b[a] * (ry.a[b] * rx.a[d]));
            }
        P.G.rowptr.push_back(int32_t(P.G.col.size()));
      }
  // D_a = G_a^T
  P.D.rowptr.assign(size_t(P.n_p) + 1, 0);
  for (int32_t q : P.G.col) ++P.D.rowptr[size_t(q) + 1];
  for (int32_t q = 0; q < P.n_p; ++q) P.D.rowptr[size_t(q) + 1] += P.D.rowptr[size_t(q)];
  P.D.col.resize(P.G.col.size());
  for (auto& v : P.Dv) v.resize(P.G.col.size());
  std::vector<int32_t> fill(P.D.rowptr.begin(), P.D.rowptr.end() - 1);
  for (int32_t r = 0; r < P.n_v; ++r)
    for (int32_t t = P.G.rowptr[size_t(r)]; t < P.G.rowptr[size_t(r) + 1]; ++t) {
      const int32_t pos = fill[size_t(P.G.col[size_t(t)])]++;
      P.D.col[size_t(pos)] = r;
      for (int a = 0; a < 3; ++a) P.Dv[a][size_t(pos)] = P.Gv[a][size_t(t)];
    }
  // pressure lumped mass
  const P1 PX = p1_matrices(xp[0]), PY = p1_matrices(xp[1]), PZ = p1_matrices(xp[2]);
  P.m_p.resize(size_t(P.n_p));
  for (int32_t k = 0; k < npz; ++k)
    for (int32_t j = 0; j < npy; ++j)
      for (int32_t i = 0; i < npx; ++i)
        P.m_p[size_t((k * npy + j) * npx + i)] = PZ.m[size_t(k)] * (PY.m[size_t(j)] * PX.m[size_t(i)]);
  // pressure hierarchy: coarsest first
  std::vector<std::array<std::vector<double>, 3>> coords(size_t(c.n_levels));
  coords.back() = xp;
  for (int l = c.n_levels - 2; l >= 0; --l)
    for (int a = 0; a < 3; ++a) coords[size_t(l)][size_t(a)] = every_other(coords[size_t(l) + 1][size_t(a)]);
  P.levels.resize(size_t(c.n_levels));
  for (int l = 0; l < c.n_levels; ++l) {
    pressure_operator(coords[size_t(l)], P.levels[size_t(l)]);
    if (l > 0) pressure_prolongation(coords[size_t(l) - 1], coords[size_t(l)], P.levels[size_t(l)]);
  }
}

}  // namespace

extern "C" {

int mgns_build(const mgns_config* cfg, mgns_problem** out) {
  try {
    if (!cfg || !out) throw Fail(MGGEN_EINVAL, "null argument");
    *out = nullptr;
    if (cfg->n_levels < 1 || cfg->n_levels > 12) throw Fail(MGGEN_EINVAL, "n_levels out of range");
    for (int a = 0; a < 3; ++a) {
      if (cfg->cells[a] < 1 || cfg->cells[a] > 4096) throw Fail(MGGEN_EINVAL, "cells out of range");
      if (cfg->cells[a] % (1 << (cfg->n_levels - 1)) != 0)
        throw Fail(MGGEN_EINVAL, "cells must be divisible by 2^(n_levels - 1)");
      if (!(cfg->length[a] > 0.0)) throw Fail(MGGEN_EINVAL, "lengths must be positive");
    }
    const int64_t nv = (2 * int64_t(cfg->cells[0]) + 1) * (2 * int64_t(cfg->cells[1]) + 1) *
                       (2 * int64_t(cfg->cells[2]) + 1);
    if (nv * 27 > INT32_MAX) throw Fail(MGGEN_EINVAL, "velocity matrices exceed 2^31 - 1 entries");
    auto* p = new mgns_problem();
    p->cfg = *cfg;
    try {
      build(*p);
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
    return MGGEN_OK;
  } catch (const Fail& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return MGGEN_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return MGGEN_EINTERNAL;
  }
}

int mgns_operators(const mgns_problem* p, mgns_view* o) {
  if (!p || !o) {
    g_err = "null argument";
    return MGGEN_EINVAL;
  }
  o->n_v = p->n_v;
  o->n_p = p->n_p;
  o->v_nnz = int64_t(p->V.col.size());
  o->V_rowptr = p->V.rowptr.data();
  o->V_col = p->V.col.data();
  o->K_val = p->K.data();
  o->g_nnz = int64_t(p->G.col.size());
  o->G_rowptr = p->G.rowptr.data();
  o->G_col = p->G.col.data();
  o->d_nnz = int64_t(p->D.col.size());
  o->D_rowptr = p->D.rowptr.data();
  o->D_col = p->D.col.data();
  for (int a = 0; a < 3; ++a) {
    o->C_val[a] = p->C[a].data();
    o->G_val[a] = p->Gv[a].data();
    o->D_val[a] = p->Dv[a].data();
  }
  o->m_v = p->m_v.data();
  o->m_p = p->m_p.data();
  o->dir_mask = p->dir_mask.data();
  o->dir_val = p->dir_val.data();
  o->coords_v = p->coords.data();
  return MGGEN_OK;
}

int32_t mgns_num_levels(const mgns_problem* p) { return p ? int32_t(p->levels.size()) : 0; }

int mgns_pressure_level(const mgns_problem* p, int32_t level, mggen_level_view* o) {
  if (!p || !o || level < 0 || level >= int32_t(p->levels.size())) {
    g_err = "bad problem, level or output";
    return MGGEN_EINVAL;
  }
  const PLevel& L = p->levels[size_t(level)];
  *o = mggen_level_view{};
  o->n_nodes = L.n;
  o->block = 1;
  o->nnzb = int64_t(L.A.col.size());
  o->rowptr = L.A.rowptr.data();
  o->col = L.A.col.data();
  o->val = L.a.data();
  o->p_cols = level > 0 ? L.p_cols : 0;
  o->p_nnz = level > 0 ? int64_t(L.P.col.size()) : 0;
  o->p_rowptr = level > 0 ? L.P.rowptr.data() : nullptr;
  o->p_col = level > 0 ? L.P.col.data() : nullptr;
  o->p_val = level > 0 ? L.p.data() : nullptr;
  o->dof_mask = L.mask.data();
  return MGGEN_OK;
}

void mgns_free(mgns_problem* p) { delete p; }

const char* mgns_last_error(void) { return g_err.c_str(); }

}  // extern "C"
