// Native problem generator: adaptive Q1 meshes, hanging nodes, global coarsening,
// constrained nodal-block operators and dyadic prolongations (host C++17 + OpenMP).
//
// Paper: Sec. 2.1 (equal-order Q^r elements, nodal blocks), Sec. 2.2 (local refinement
// with one level jump, hanging nodes through H, global coarsening), Sec. 4.1 "Geometric
// Multigrid CUDA" (prolongation from element-local coefficients, R = P^T).
//
// Tree representation: for every depth j a byte map over the depth-j cell grid says
// whether that cell is refined.  A cell exists when its parent is refined; a leaf is an
// existing cell that is not refined.  The one-level-jump rule is enforced in its
// "ripple" form: every refined cell at depth j needs all of its vertex neighbours at
// depth j to exist (equivalent to "no leaf touches a leaf two or more levels deeper").
#include "../../../include/mggen.h"

#include <omp.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
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

// ---------------------------------------------------------------- tree
struct Tree {
  int dim = 2, D = 0;
  int64_t nc[3] = {1, 1, 1};
  double h0 = 1.0;
  std::vector<std::vector<uint8_t>> ref;   // ref[j][cell] for j = 0..D

  int64_t n(int j, int a) const { return a < dim ? (nc[a] << j) : 1; }
  int64_t cells(int j) const { return n(j, 0) * n(j, 1) * n(j, 2); }
  int64_t cid(int j, int64_t x, int64_t y, int64_t z) const { return (z * n(j, 1) + y) * n(j, 0) + x; }
  bool inside(int j, int64_t x, int64_t y, int64_t z) const {
    return x >= 0 && y >= 0 && z >= 0 && x < n(j, 0) && y < n(j, 1) && z < n(j, 2);
  }
  bool exists(int j, int64_t x, int64_t y, int64_t z) const {
    return j == 0 || ref[j - 1][cid(j - 1, x >> 1, y >> 1, z >> 1)];
  }
  bool refined(int j, int64_t x, int64_t y, int64_t z) const { return ref[j][cid(j, x, y, z)] != 0; }
  double hf() const { return h0 / double(int64_t(1) << D); }
  int64_t vn(int a) const { return a < dim ? (nc[a] << D) + 1 : 1; }   // vertex lattice extent
  int64_t vid(int64_t x, int64_t y, int64_t z) const { return (z * vn(1) + y) * vn(0) + x; }
  void init(int d, const int32_t* c, double h, int depth) {
    dim = d;
    D = depth;
    for (int a = 0; a < 3; ++a) nc[a] = a < d ? c[a] : 1;
    h0 = h;
    ref.assign(D + 1, {});
    for (int j = 0; j <= D; ++j) ref[j].assign(cells(j), 0);
  }
  template <class F> void for_each_leaf(F&& f) const {   // by depth, then lexicographic
    for (int j = 0; j <= D; ++j)
      for (int64_t z = 0; z < n(j, 2); ++z)
        for (int64_t y = 0; y < n(j, 1); ++y)
          for (int64_t x = 0; x < n(j, 0); ++x)
            if (exists(j, x, y, z) && !refined(j, x, y, z)) f(j, x, y, z);
  }
  int max_leaf_depth() const {
    int m = 0;
    for_each_leaf([&](int j, int64_t, int64_t, int64_t) { m = std::max(m, j); });
    return m;
  }
};

struct Cell { int j; int64_t x, y, z; };

void balance(Tree& t) {
  const int d3 = t.dim == 3;
  bool changed = true;
  while (changed) {
    changed = false;
    for (int j = t.D - 1; j >= 1; --j) {
      for (int64_t z = 0; z < t.n(j, 2); ++z)
        for (int64_t y = 0; y < t.n(j, 1); ++y)
          for (int64_t x = 0; x < t.n(j, 0); ++x) {
            if (!t.refined(j, x, y, z) || !t.exists(j, x, y, z)) continue;
            for (int dz = -d3; dz <= d3; ++dz)
              for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                  int64_t qx = x + dx, qy = y + dy, qz = z + dz;
                  if (!t.inside(j, qx, qy, qz) || t.exists(j, qx, qy, qz)) continue;
                  // refine the leaf that covers the missing neighbour position
                  for (int k = j - 1; k >= 0; --k) {
                    int sh = j - k;
                    int64_t cx = qx >> sh, cy = qy >> sh, cz = qz >> sh;
                    if (t.exists(k, cx, cy, cz)) {
                      if (t.refined(k, cx, cy, cz)) throw Fail(MGGEN_EINTERNAL, "balance: inconsistent tree");
                      t.ref[k][t.cid(k, cx, cy, cz)] = 1;
                      changed = true;
                      break;
                    }
                  }
                }
          }
    }
  }
}

void apply_round(Tree& t, const mggen_round& r) {
  std::vector<Cell> mark;
  const double hf = t.hf();
  const int dmax = t.max_leaf_depth();
  t.for_each_leaf([&](int j, int64_t x, int64_t y, int64_t z) {
    const int64_t s = int64_t(1) << (t.D - j);
    bool hit = false;
    if (r.kind == MGGEN_ROUND_UNIFORM) {
      hit = true;
    } else if (r.kind == MGGEN_ROUND_BAND) {
      const double cx = r.p[0], cy = r.p[1], rad = r.p[2], del = r.p[3];
      const double x0 = double(x * s) * hf, x1 = double(x * s + s) * hf;
      const double y0 = double(y * s) * hf, y1 = double(y * s + s) * hf;
      const double nx = std::min(std::max(cx, x0), x1) - cx;
      const double ny = std::min(std::max(cy, y0), y1) - cy;
      const double dmin2 = nx * nx + ny * ny;
      const double fx = std::max(std::fabs(x0 - cx), std::fabs(x1 - cx));
      const double fy = std::max(std::fabs(y0 - cy), std::fabs(y1 - cy));
      const double dmax2 = fx * fx + fy * fy;
      const double ro = rad + del, ri = rad - del;
      hit = ri > 0 ? (dmin2 < ro * ro && dmax2 > ri * ri) : (dmin2 < ro * ro);
    } else if (r.kind == MGGEN_ROUND_CORNER) {
      if (j == dmax) {
        hit = true;
        const int64_t lo[3] = {x, y, z};
        for (int a = 0; a < t.dim; ++a)
          if (r.axes >> a & 1) hit = hit && (double((lo[a] + 1) * s) * hf <= r.p[0]);
      }
    } else {
      throw Fail(MGGEN_EINVAL, "unknown refinement rule");
    }
    if (hit) mark.push_back({j, x, y, z});
  });
  for (const Cell& c : mark) {
    if (c.j >= t.D) throw Fail(MGGEN_EINVAL, "refinement beyond the lattice depth");
    t.ref[c.j][t.cid(c.j, c.x, c.y, c.z)] = 1;
  }
  balance(t);
}

// One global coarsening step: families whose children are all leaves are coarsened
// together, except those whose coarsening would leave a refined vertex neighbour of one
// of their children without that child (dropped until nothing changes).
Tree coarsen(const Tree& t) {
  const int d3 = t.dim == 3;
  std::vector<std::vector<uint8_t>> cand(t.D + 1);
  for (int k = 0; k <= t.D; ++k) cand[k].assign(t.cells(k), 0);
  for (int k = 0; k < t.D; ++k)
    for (int64_t z = 0; z < t.n(k, 2); ++z)
      for (int64_t y = 0; y < t.n(k, 1); ++y)
        for (int64_t x = 0; x < t.n(k, 0); ++x) {
          if (!t.exists(k, x, y, z) || !t.refined(k, x, y, z)) continue;
          bool leafkids = true;
          for (int oz = 0; oz <= d3; ++oz)
            for (int oy = 0; oy < 2; ++oy)
              for (int ox = 0; ox < 2; ++ox)
                leafkids = leafkids && !t.refined(k + 1, 2 * x + ox, 2 * y + oy, 2 * z + oz);
          if (leafkids) cand[k][t.cid(k, x, y, z)] = 1;
        }
  bool dropped = true;
  while (dropped) {
    dropped = false;
    for (int k = 0; k < t.D; ++k) {
      const int c = k + 1;   // depth of the children
      for (int64_t z = 0; z < t.n(k, 2); ++z)
        for (int64_t y = 0; y < t.n(k, 1); ++y)
          for (int64_t x = 0; x < t.n(k, 0); ++x) {
            if (!cand[k][t.cid(k, x, y, z)]) continue;
            bool bad = false;
            for (int oz = 0; oz <= d3 && !bad; ++oz)
              for (int oy = 0; oy < 2 && !bad; ++oy)
                for (int ox = 0; ox < 2 && !bad; ++ox) {
                  const int64_t qx = 2 * x + ox, qy = 2 * y + oy, qz = 2 * z + oz;
                  for (int dz = -d3; dz <= d3 && !bad; ++dz)
                    for (int dy = -1; dy <= 1 && !bad; ++dy)
                      for (int dx = -1; dx <= 1 && !bad; ++dx) {
                        const int64_t px = qx + dx, py = qy + dy, pz = qz + dz;
                        if (!t.inside(c, px, py, pz) || !t.exists(c, px, py, pz)) continue;
                        if (t.refined(c, px, py, pz) && !cand[c][t.cid(c, px, py, pz)]) bad = true;
                      }
                }
            if (bad) {
              cand[k][t.cid(k, x, y, z)] = 0;
              dropped = true;
            }
          }
    }
  }
  Tree out = t;
  for (int k = 0; k <= t.D; ++k)
    for (size_t i = 0; i < cand[k].size(); ++i)
      if (cand[k][i]) out.ref[k][i] = 0;
  // cells below a coarsened family no longer exist; clear stale flags for clarity
  for (int k = 1; k <= t.D; ++k)
    for (int64_t z = 0; z < out.n(k, 2); ++z)
      for (int64_t y = 0; y < out.n(k, 1); ++y)
        for (int64_t x = 0; x < out.n(k, 0); ++x)
          if (!out.exists(k, x, y, z)) out.ref[k][out.cid(k, x, y, z)] = 0;
  return out;
}

// ---------------------------------------------------------------- mesh of one level
struct Leaf { int j; int64_t a[3]; int64_t s; };

struct MeshLevel {
  int dim = 2;
  std::vector<Leaf> leaves;
  std::vector<int32_t> node_of_v;          // vertex lattice -> node id (-1)
  std::vector<int32_t> lat;                // node -> lattice coords (x, y, z)
  int32_t n = 0;
  std::vector<int32_t> corner;             // leaves * nb
  std::vector<uint8_t> hanging;            // per node
  std::vector<int32_t> hmaster;            // per node * 4 (-1)
  std::vector<double> hweight;             // per node * 4
  std::vector<int32_t> hang_list;
};

MeshLevel make_mesh(const Tree& t) {
  MeshLevel m;
  m.dim = t.dim;
  const int nb = 1 << t.dim;
  t.for_each_leaf([&](int j, int64_t x, int64_t y, int64_t z) {
    const int64_t s = int64_t(1) << (t.D - j);
    m.leaves.push_back({j, {x * s, y * s, z * s}, s});
  });
  const int64_t nv = t.vn(0) * t.vn(1) * t.vn(2);
  std::vector<uint8_t> isnode(nv, 0);
  for (const Leaf& L : m.leaves)
    for (int c = 0; c < nb; ++c)
      isnode[t.vid(L.a[0] + (c & 1) * L.s, L.a[1] + (c >> 1 & 1) * L.s,
                   t.dim == 3 ? L.a[2] + (c >> 2 & 1) * L.s : 0)] = 1;
  m.node_of_v.assign(nv, -1);
  int32_t cnt = 0;
  for (int64_t v = 0; v < nv; ++v)
    if (isnode[v]) m.node_of_v[v] = cnt++;
  m.n = cnt;
  m.lat.resize(size_t(cnt) * 3);
  for (int64_t z = 0; z < t.vn(2); ++z)
    for (int64_t y = 0; y < t.vn(1); ++y)
      for (int64_t x = 0; x < t.vn(0); ++x) {
        int32_t id = m.node_of_v[t.vid(x, y, z)];
        if (id >= 0) {
          m.lat[3 * id] = int32_t(x);
          m.lat[3 * id + 1] = int32_t(y);
          m.lat[3 * id + 2] = int32_t(z);
        }
      }
  m.corner.resize(m.leaves.size() * nb);
  for (size_t e = 0; e < m.leaves.size(); ++e) {
    const Leaf& L = m.leaves[e];
    for (int c = 0; c < nb; ++c)
      m.corner[e * nb + c] = m.node_of_v[t.vid(L.a[0] + (c & 1) * L.s, L.a[1] + (c >> 1 & 1) * L.s,
                                               t.dim == 3 ? L.a[2] + (c >> 2 & 1) * L.s : 0)];
  }
  // hanging nodes: edge midpoints and face centres of leaves that are mesh nodes
  m.hanging.assign(cnt, 0);
  m.hmaster.assign(size_t(cnt) * 4, -1);
  m.hweight.assign(size_t(cnt) * 4, 0.0);
  auto node_at = [&](const int64_t p[3]) { return m.node_of_v[t.vid(p[0], p[1], t.dim == 3 ? p[2] : 0)]; };
  auto record = [&](const int64_t p[3], const int64_t (*ms)[3], int k, double w) {
    int32_t h = node_at(p);
    if (h < 0) return;
    int32_t mm[4];
    for (int q = 0; q < k; ++q) {
      mm[q] = node_at(ms[q]);
      if (mm[q] < 0) throw Fail(MGGEN_EINTERNAL, "master of a hanging node is not a node");
    }
    if (m.hanging[h]) {
      for (int q = 0; q < k; ++q)
        if (m.hmaster[4 * h + q] != mm[q]) throw Fail(MGGEN_EINTERNAL, "inconsistent hanging masters");
      return;
    }
    m.hanging[h] = 1;
    for (int q = 0; q < k; ++q) {
      m.hmaster[4 * h + q] = mm[q];
      m.hweight[4 * h + q] = w;
    }
  };
  for (const Leaf& L : m.leaves) {
    if (L.s < 2) continue;
    const int64_t h = L.s / 2;
    for (int a = 0; a < t.dim; ++a) {
      int oth[2], no = 0;
      for (int b = 0; b < t.dim; ++b)
        if (b != a) oth[no++] = b;
      for (int o = 0; o < (1 << no); ++o) {
        int64_t p[3] = {L.a[0], L.a[1], L.a[2]};
        for (int q = 0; q < no; ++q) p[oth[q]] += ((o >> q) & 1) * L.s;
        p[a] += h;
        int64_t ms[2][3];
        for (int q = 0; q < 3; ++q) ms[0][q] = ms[1][q] = p[q];
        ms[0][a] -= h;
        ms[1][a] += h;
        record(p, ms, 2, 0.5);
      }
    }
    if (t.dim == 3) {
      for (int nax = 0; nax < 3; ++nax) {
        int t0 = nax == 0 ? 1 : 0, t1 = nax == 2 ? 1 : 2;
        for (int o = 0; o < 2; ++o) {
          int64_t p[3] = {L.a[0], L.a[1], L.a[2]};
          p[nax] += o * L.s;
          p[t0] += h;
          p[t1] += h;
          int64_t ms[4][3];
          const int64_t sg[4][2] = {{-h, -h}, {-h, h}, {h, -h}, {h, h}};
          for (int q = 0; q < 4; ++q) {
            for (int r = 0; r < 3; ++r) ms[q][r] = p[r];
            ms[q][t0] += sg[q][0];
            ms[q][t1] += sg[q][1];
          }
          record(p, ms, 4, 0.25);
        }
      }
    }
  }
  for (int32_t i = 0; i < cnt; ++i)
    if (m.hanging[i]) {
      m.hang_list.push_back(i);
      for (int q = 0; q < 4; ++q) {
        int32_t mm = m.hmaster[4 * i + q];
        if (mm >= 0 && m.hanging[mm]) throw Fail(MGGEN_EINTERNAL, "a master of a hanging node is hanging");
      }
    }
  return m;
}

// ---------------------------------------------------------------- element matrices
// 1D reference matrices on [0, s]: stiffness, mass, and int phi_i phi_j' (scale free)
inline double k1(int i, int j, double s) { return (i == j ? 1.0 : -1.0) / s; }
inline double m1(int i, int j, double s) { return (i == j ? 2.0 : 1.0) * s / 6.0; }
inline double g1(int, int j) { return j ? 0.5 : -0.5; }

double langevin(double pe) {
  if (pe < 1e-2) return pe / 3.0 - pe * pe * pe / 45.0 + 2.0 * std::pow(pe, 5) / 945.0;
  return 1.0 / std::tanh(pe) - 1.0 / pe;
}

double supg_tau(const mggen_config& c, double s) {
  const double bx = c.bvec[0], by = c.bvec[1];
  const double nb = std::sqrt(bx * bx + by * by);
  if (nb == 0.0 || c.no_supg) return 0.0;
  const double hk = s * nb / std::max(std::fabs(bx), std::fabs(by));
  const double pe = nb * hk / (2.0 * c.eps);
  return hk / (2.0 * nb) * langevin(pe);
}

// d_{km}[a][b] = int d_k phi_a d_m phi_b over a box of side s (tensor products)
double dd(int dim, int k, int m, int a, int b, double s) {
  double v = 1.0;
  for (int ax = 0; ax < dim; ++ax) {
    const int ia = (a >> ax) & 1, ib = (b >> ax) & 1;
    if (ax == k && ax == m) v *= k1(ia, ib, s);
    else if (ax == k) v *= g1(ib, ia);        // int phi_a' phi_b
    else if (ax == m) v *= g1(ia, ib);        // int phi_a phi_b'
    else v *= m1(ia, ib, s);
  }
  return v;
}

// int phi_a (d_k phi_b)
double gradtrial(int dim, int k, int a, int b, double s) {
  double v = 1.0;
  for (int ax = 0; ax < dim; ++ax) {
    const int ia = (a >> ax) & 1, ib = (b >> ax) & 1;
    v *= ax == k ? g1(ia, ib) : m1(ia, ib, s);
  }
  return v;
}

void beta_at(const mggen_config& c, const double x[3], double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  for (int k = 0; k < 8; ++k) {
    double e[3] = {0, 0, 0};
    e[c.j[k]] = 1.0;
    const double* kp = c.kappa[k];
    const double cr[3] = {kp[1] * e[2] - kp[2] * e[1], kp[2] * e[0] - kp[0] * e[2], kp[0] * e[1] - kp[1] * e[0]};
    const double ang = 2.0 * kPi * (x[0] * kp[0] + x[1] * kp[1] + x[2] * kp[2]) + c.phi[k];
    const double f = c.a[k] * 2.0 * kPi * std::cos(ang);
    for (int q = 0; q < 3; ++q) out[q] += f * cr[q];
  }
  for (int q = 0; q < 3; ++q) out[q] *= c.scale;
}

struct Gauss { int n; double p[3], w[3]; };
Gauss gauss(int n) {
  Gauss g{};
  g.n = n;
  if (n == 2) {
    const double q = 0.5 / std::sqrt(3.0);
    g.p[0] = 0.5 - q; g.p[1] = 0.5 + q; g.w[0] = g.w[1] = 0.5;
  } else {
    const double q = 0.5 * std::sqrt(0.6);
    g.p[0] = 0.5 - q; g.p[1] = 0.5; g.p[2] = 0.5 + q;
    g.w[0] = 5.0 / 18.0; g.w[1] = 8.0 / 18.0; g.w[2] = 5.0 / 18.0;
  }
  return g;
}

// row `a` of the element matrix of the PDE's bilinear form on a box (lower corner x0,
// side s): out[b][ci][cj]
void element_row_pde(const mggen_config& c, int a, double s, const double x0[3], double* out) {
  const int dim = c.dim, nb = 1 << dim, B = c.block;
  std::fill(out, out + nb * B * B, 0.0);
  if (c.pde == MGGEN_PDE_POISSON || c.pde == MGGEN_PDE_TD) {
    double tau = c.pde == MGGEN_PDE_TD ? supg_tau(c, s) : 0.0;
    for (int b = 0; b < nb; ++b) {
      double lap = 0.0;
      for (int k = 0; k < dim; ++k) lap += dd(dim, k, k, a, b, s);
      if (c.pde == MGGEN_PDE_POISSON) { out[b] = lap; continue; }
      double conv = 0.0, stab = 0.0;
      for (int k = 0; k < dim; ++k) conv += c.bvec[k] * gradtrial(dim, k, a, b, s);
      for (int k = 0; k < dim; ++k)
        for (int m = 0; m < dim; ++m) stab += c.bvec[k] * c.bvec[m] * dd(dim, m, k, a, b, s);
      out[b] = c.eps * lap + conv + tau * stab;
    }
    return;
  }
  if (c.pde == MGGEN_PDE_ELASTICITY) {
    for (int b = 0; b < nb; ++b) {
      double lap = 0.0;
      for (int k = 0; k < dim; ++k) lap += dd(dim, k, k, a, b, s);
      for (int ci = 0; ci < dim; ++ci)
        for (int cj = 0; cj < dim; ++cj) {
          double v = c.mu * dd(dim, cj, ci, a, b, s) + c.lam * dd(dim, ci, cj, a, b, s);
          if (ci == cj) v += c.mu * lap;
          out[(b * B + ci) * B + cj] = v;
        }
    }
    return;
  }
  if (c.pde == MGGEN_PDE_OSEEN) {
    // 2-point Gauss per direction with beta at the points; delta_K with beta at the centre
    const Gauss g = gauss(2);
    const double xc[3] = {x0[0] + 0.5 * s, x0[1] + 0.5 * s, x0[2] + 0.5 * s};
    double bc[3];
    beta_at(c, xc, bc);
    const double bn = std::sqrt(bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
    const double delta = c.pspg_alpha / (c.nu / (s * s) + bn / s + 1.0 / c.dt);
    const double jac = s * s * s;
    for (int qz = 0; qz < 2; ++qz)
      for (int qy = 0; qy < 2; ++qy)
        for (int qx = 0; qx < 2; ++qx) {
          const double xi[3] = {g.p[qx], g.p[qy], g.p[qz]};
          const double w = g.w[qx] * g.w[qy] * g.w[qz] * jac;
          const double xq[3] = {x0[0] + s * xi[0], x0[1] + s * xi[1], x0[2] + s * xi[2]};
          double be[3];
          beta_at(c, xq, be);
          double phi[8], grad[8][3];
          for (int q = 0; q < 8; ++q) {
            double h[3], dh[3];
            for (int k = 0; k < 3; ++k) {
              const int o = (q >> k) & 1;
              h[k] = o ? xi[k] : 1.0 - xi[k];
              dh[k] = (o ? 1.0 : -1.0) / s;
            }
            phi[q] = h[0] * h[1] * h[2];
            grad[q][0] = dh[0] * h[1] * h[2];
            grad[q][1] = h[0] * dh[1] * h[2];
            grad[q][2] = h[0] * h[1] * dh[2];
          }
          for (int b = 0; b < 8; ++b) {
            const double gg = grad[b][0] * grad[a][0] + grad[b][1] * grad[a][1] + grad[b][2] * grad[a][2];
            const double bgb = be[0] * grad[b][0] + be[1] * grad[b][1] + be[2] * grad[b][2];
            double* o = out + b * 16;
            o[0] += w * delta * gg;
            for (int k = 0; k < 3; ++k) {
              o[1 + k] += w * grad[b][k] * phi[a];
              o[(1 + k) * 4] += -w * phi[b] * grad[a][k];
              o[(1 + k) * 4 + 1 + k] += w * (phi[b] * phi[a] / c.dt + c.nu * gg + bgb * phi[a]);
            }
          }
        }
    return;
  }
  throw Fail(MGGEN_EINVAL, "unknown pde");
}

// row `a` of the element matrix: the PDE's form plus, for time-dependent problems, the
// lumped mass term c M_l (eq. mass_lumping: m_i = int phi_i, each cell giving |K| / 2^dim
// to each corner), c = mass_coef
void element_row(const mggen_config& c, int a, double s, const double x0[3], double* out) {
  element_row_pde(c, a, s, x0, out);
  if (c.mass_coef != 0.0) {
    const int nb = 1 << c.dim, B = c.block;
    const double vol = c.dim == 3 ? s * s * s : s * s;
    for (int ci = 0; ci < B; ++ci) out[(a * B + ci) * B + ci] += c.mass_coef * vol / double(nb);
  }
}

// load entries of corner `a` (3-point Gauss per direction): out[ci]
void element_load(const mggen_config& c, int a, double s, const double x0[3], double* out) {
  const int dim = c.dim, B = c.block;
  std::fill(out, out + B, 0.0);
  if (c.rhs == MGGEN_RHS_NONE || c.rhs == MGGEN_RHS_NOISE) return;
  const Gauss g = gauss(3);
  const double jac = dim == 3 ? s * s * s : s * s;
  const double tau = (c.rhs == MGGEN_RHS_DISK && c.pde == MGGEN_PDE_TD) ? supg_tau(c, s) : 0.0;
  const int nz = dim == 3 ? 3 : 1;
  for (int qz = 0; qz < nz; ++qz)
    for (int qy = 0; qy < 3; ++qy)
      for (int qx = 0; qx < 3; ++qx) {
        const double xi[3] = {g.p[qx], g.p[qy], dim == 3 ? g.p[qz] : 0.0};
        const double w = g.w[qx] * g.w[qy] * (dim == 3 ? g.w[qz] : 1.0) * jac;
        double h = 1.0, grad[3] = {1, 1, 1};
        for (int k = 0; k < dim; ++k) {
          const int o = (a >> k) & 1;
          const double hk = o ? xi[k] : 1.0 - xi[k];
          const double dk = (o ? 1.0 : -1.0) / s;
          for (int m = 0; m < dim; ++m) grad[m] *= (m == k ? dk : hk);
          h *= hk;
        }
        const double xq[3] = {x0[0] + s * xi[0], x0[1] + s * xi[1], dim == 3 ? x0[2] + s * xi[2] : 0.0};
        if (c.rhs == MGGEN_RHS_SINSIN) {
          out[0] += w * (2.0 * kPi * kPi * std::sin(kPi * xq[0]) * std::sin(kPi * xq[1])) * h;
        } else if (c.rhs == MGGEN_RHS_DISK) {
          const double dx = xq[0] - 0.5, dy = xq[1] - 0.5;
          const double f = (dx * dx + dy * dy < 0.3 * 0.3) ? 1.0 : 0.0;
          out[0] += w * f * h;
          if (tau != 0.0) out[0] += tau * (w * f * (c.bvec[0] * grad[0] + c.bvec[1] * grad[1]));
        } else if (c.rhs == MGGEN_RHS_CONST) {
          for (int ci = 0; ci < B; ++ci) out[ci] += c.rhs_const[ci] * (w * h);
        } else if (c.rhs == MGGEN_RHS_FIELD) {
          double f[3] = {0, 0, 0};
          for (int m = 0; m < 4; ++m) {
            const double ang = 2.0 * kPi * (xq[0] * c.fk[m][0] + xq[1] * c.fk[m][1] + xq[2] * c.fk[m][2]) + c.fphi[m];
            f[c.fi[m]] += c.fc[m] * std::sin(ang);
          }
          for (int k = 0; k < 3; ++k) out[1 + k] += w * f[k] * h;
        }
      }
}

// ---------------------------------------------------------------- level assembly
struct LevelOut {
  int32_t n = 0, block = 1;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val;
  int32_t p_cols = 0;
  std::vector<int32_t> prow, pcol;
  std::vector<double> pval;
  std::vector<uint8_t> mask;
  std::vector<int32_t> hang_node, hang_master, lat;
  std::vector<double> hang_weight;
  int32_t max_depth = 0;
  std::vector<int32_t> cells;      // leaf corners, leaves * 2^dim (bit k of a corner = axis k)
  std::vector<double> cell_size;   // leaf edge lengths
};

struct Expand { int cnt; int32_t node[4]; double w[4]; };

inline Expand expand(const MeshLevel& m, int32_t k) {
  Expand e{};
  if (!m.hanging[k]) {
    e.cnt = 1; e.node[0] = k; e.w[0] = 1.0;
  } else {
    for (int q = 0; q < 4; ++q)
      if (m.hmaster[4 * k + q] >= 0) { e.node[e.cnt] = m.hmaster[4 * k + q]; e.w[e.cnt] = m.hweight[4 * k + q]; ++e.cnt; }
  }
  return e;
}

void assemble(const mggen_config& c, const Tree& t, const MeshLevel& m, LevelOut& L, std::vector<double>* rhs) {
  const int dim = c.dim, nb = 1 << dim, B = c.block;
  const int32_t n = m.n;
  const size_t ne = m.leaves.size();
  L.n = n;
  L.block = B;
  // constrained components
  L.mask.assign(size_t(n) * B, 0);
  for (int32_t i = 0; i < n; ++i) {
    if (m.hanging[i]) for (int ci = 0; ci < B; ++ci) L.mask[size_t(i) * B + ci] = 1;
    bool on = false;
    for (int a = 0; a < dim; ++a) {
      const int64_t top = t.nc[a] << t.D;
      if ((c.dir_faces >> (2 * a) & 1) && m.lat[3 * i + a] == 0) on = true;
      if ((c.dir_faces >> (2 * a + 1) & 1) && m.lat[3 * i + a] == top) on = true;
    }
    if (on) for (int ci = 0; ci < B; ++ci) if (c.dir_comps >> ci & 1) L.mask[size_t(i) * B + ci] = 1;
  }
  std::vector<uint8_t> free_node(n, 0);
  for (int32_t i = 0; i < n; ++i)
    for (int ci = 0; ci < B; ++ci) free_node[i] |= !L.mask[size_t(i) * B + ci];
  // U(e): regular nodes reached by the corners of leaf e through H
  std::vector<int32_t> uptr(ne + 1, 0), unodes;
  {
    std::vector<int32_t> tmp;
    for (size_t e = 0; e < ne; ++e) {
      tmp.clear();
      for (int a = 0; a < nb; ++a) {
        Expand x = expand(m, m.corner[e * nb + a]);
        for (int q = 0; q < x.cnt; ++q) tmp.push_back(x.node[q]);
      }
      std::sort(tmp.begin(), tmp.end());
      tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
      unodes.insert(unodes.end(), tmp.begin(), tmp.end());
      uptr[e + 1] = int32_t(unodes.size());
    }
  }
  // incidence: node -> leaves whose U contains it (in leaf order)
  std::vector<int32_t> iptr(size_t(n) + 1, 0), ileaf(unodes.size());
  for (int32_t u : unodes) ++iptr[u + 1];
  for (int32_t i = 0; i < n; ++i) iptr[i + 1] += iptr[i];
  {
    std::vector<int32_t> fill(iptr.begin(), iptr.end() - 1);
    for (size_t e = 0; e < ne; ++e)
      for (int32_t k = uptr[e]; k < uptr[e + 1]; ++k) ileaf[fill[unodes[k]]++] = int32_t(e);
  }
  // block pattern per row
  std::vector<std::vector<int32_t>> rows(n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t i = 0; i < n; ++i) {
    std::vector<int32_t>& r = rows[i];
    if (free_node[i]) {
      for (int32_t k = iptr[i]; k < iptr[i + 1]; ++k) {
        const int32_t e = ileaf[k];
        for (int32_t q = uptr[e]; q < uptr[e + 1]; ++q) {
          const int32_t j = unodes[q];
          if (j == i || free_node[j]) r.push_back(j);
        }
      }
    }
    r.push_back(i);
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
  }
  L.rowptr.assign(size_t(n) + 1, 0);
  for (int32_t i = 0; i < n; ++i) L.rowptr[i + 1] = L.rowptr[i] + int32_t(rows[i].size());
  const int64_t nnzb = L.rowptr[n];
  if (nnzb >= (int64_t(1) << 31)) throw Fail(MGGEN_EINVAL, "too many blocks for int32 indices");
  L.col.resize(nnzb);
  L.val.assign(size_t(nnzb) * B * B, 0.0);
  const double hf = t.hf();
  const bool per_depth = c.pde != MGGEN_PDE_OSEEN;
  // element rows per depth for the constant-coefficient operators
  std::vector<std::vector<double>> kdepth(t.D + 1);
  if (per_depth) {
    for (int j = 0; j <= t.D; ++j) {
      kdepth[j].resize(size_t(nb) * nb * B * B);
      const double s = hf * double(int64_t(1) << (t.D - j));
      const double x0[3] = {0, 0, 0};
      for (int a = 0; a < nb; ++a) element_row(c, a, s, x0, &kdepth[j][size_t(a) * nb * B * B]);
    }
  }
  if (rhs) rhs->assign(size_t(n) * B, 0.0);
#pragma omp parallel
  {
    std::vector<double> krow(size_t(nb) * B * B), frow(B);
#pragma omp for schedule(dynamic, 512)
    for (int32_t i = 0; i < n; ++i) {
      const std::vector<int32_t>& r = rows[i];
      const int32_t base = L.rowptr[i];
      std::copy(r.begin(), r.end(), L.col.begin() + base);
      double* vrow = &L.val[size_t(base) * B * B];
      double* brow = rhs ? &(*rhs)[size_t(i) * B] : nullptr;
      if (free_node[i]) {
        for (int32_t k = iptr[i]; k < iptr[i + 1]; ++k) {
          const int32_t e = ileaf[k];
          const Leaf& Lf = m.leaves[e];
          const double s = hf * double(Lf.s);
          const double x0[3] = {double(Lf.a[0]) * hf, double(Lf.a[1]) * hf, double(Lf.a[2]) * hf};
          for (int a = 0; a < nb; ++a) {
            const Expand ea = expand(m, m.corner[size_t(e) * nb + a]);
            double wa = 0.0;
            for (int q = 0; q < ea.cnt; ++q)
              if (ea.node[q] == i) wa += ea.w[q];
            if (wa == 0.0) continue;
            const double* kr;
            if (per_depth) {
              kr = &kdepth[Lf.j][size_t(a) * nb * B * B];
            } else {
              element_row(c, a, s, x0, krow.data());
              kr = krow.data();
            }
            for (int b = 0; b < nb; ++b) {
              const Expand eb = expand(m, m.corner[size_t(e) * nb + b]);
              for (int q = 0; q < eb.cnt; ++q) {
                const int32_t j = eb.node[q];
                auto it = std::lower_bound(r.begin(), r.end(), j);
                if (it == r.end() || *it != j) continue;   // constrained column node
                double* blk = vrow + size_t(it - r.begin()) * B * B;
                const double w = wa * eb.w[q];
                const double* kb = kr + size_t(b) * B * B;
                for (int z = 0; z < B * B; ++z) blk[z] += w * kb[z];
              }
            }
            if (brow) {
              element_load(c, a, s, x0, frow.data());
              for (int ci = 0; ci < B; ++ci) brow[ci] += wa * frow[ci];
            }
          }
        }
      }
      // mask rows and columns of constrained components; identity on their diagonal
      for (size_t q = 0; q < r.size(); ++q) {
        const int32_t j = r[q];
        double* blk = vrow + q * B * B;
        for (int ci = 0; ci < B; ++ci)
          for (int cj = 0; cj < B; ++cj) {
            const bool mr = L.mask[size_t(i) * B + ci], mc = L.mask[size_t(j) * B + cj];
            if (mr || mc) blk[ci * B + cj] = (i == j && ci == cj && mr) ? 1.0 : 0.0;
          }
      }
      if (brow)
        for (int ci = 0; ci < B; ++ci)
          if (L.mask[size_t(i) * B + ci]) brow[ci] = 0.0;
    }
  }
  L.hang_node = m.hang_list;
  for (int32_t h : m.hang_list)
    for (int q = 0; q < 4; ++q) {
      L.hang_master.push_back(m.hmaster[4 * h + q]);
      L.hang_weight.push_back(m.hweight[4 * h + q]);
    }
  L.lat = m.lat;
  L.cells = m.corner;
  L.cell_size.resize(ne);
  for (size_t e = 0; e < ne; ++e) L.cell_size[e] = hf * double(m.leaves[e].s);
}

// P~ = Q H_coarse: coarse nodal basis at the fine nodes, hanging coarse corners expanded
void prolongation(const Tree& tf, const MeshLevel& mf, const Tree& tc, const MeshLevel& mc, LevelOut& L) {
  const int dim = tf.dim, nb = 1 << dim;
  const int32_t n = mf.n;
  std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t i = 0; i < n; ++i) {
    const int64_t p[3] = {mf.lat[3 * i], mf.lat[3 * i + 1], mf.lat[3 * i + 2]};
    int64_t cell[3];
    for (int a = 0; a < 3; ++a) cell[a] = a < dim ? std::min<int64_t>(p[a], (tc.nc[a] << tc.D) - 1) : 0;
    int j = 0;
    while (true) {
      const int sh = tc.D - j;
      const int64_t cx = cell[0] >> sh, cy = cell[1] >> sh, cz = cell[2] >> sh;
      if (!tc.refined(j, cx, cy, cz)) break;
      ++j;
    }
    const int64_t s = int64_t(1) << (tc.D - j);
    int64_t anc[3];
    for (int a = 0; a < 3; ++a) anc[a] = (cell[a] / s) * s;
    std::vector<std::pair<int32_t, double>> acc;
    for (int c = 0; c < nb; ++c) {
      double w = 1.0;
      int64_t cp[3] = {anc[0], anc[1], anc[2]};
      for (int a = 0; a < dim; ++a) {
        const int o = (c >> a) & 1;
        const double tt = double(p[a] - anc[a]) / double(s);
        w *= o ? tt : 1.0 - tt;
        cp[a] += o * s;
      }
      const int32_t cn = mc.node_of_v[tc.vid(cp[0], cp[1], dim == 3 ? cp[2] : 0)];
      if (cn < 0) throw Fail(MGGEN_EINTERNAL, "coarse corner is not a node");
      const Expand ex = expand(mc, cn);
      for (int q = 0; q < ex.cnt; ++q) {
        const double v = w * ex.w[q];
        bool found = false;
        for (auto& pr : acc)
          if (pr.first == ex.node[q]) { pr.second += v; found = true; break; }
        if (!found) acc.push_back({ex.node[q], v});
      }
    }
    std::vector<std::pair<int32_t, double>>& r = rows[i];
    for (auto& pr : acc)
      if (pr.second != 0.0) r.push_back(pr);
    std::sort(r.begin(), r.end());
  }
  L.p_cols = mc.n;
  L.prow.assign(size_t(n) + 1, 0);
  for (int32_t i = 0; i < n; ++i) L.prow[i + 1] = L.prow[i] + int32_t(rows[i].size());
  L.pcol.resize(L.prow[n]);
  L.pval.resize(L.prow[n]);
  for (int32_t i = 0; i < n; ++i)
    for (size_t q = 0; q < rows[i].size(); ++q) {
      L.pcol[L.prow[i] + q] = rows[i][q].first;
      L.pval[L.prow[i] + q] = rows[i][q].second;
    }
}

}  // namespace

// right-hand-side operators of a time-stepping run on the finest level
struct TimeOps {
  int32_t n_dofs = 0, n_g = 0;
  std::vector<int32_t> rrow, rcol, hrow, hcol, gidx;
  std::vector<double> rval, hval, coords;
};

namespace {

// R = [Z H^T M_l | -Z H^T A_full E_g], H at DoF level, Dirichlet DoF list, coordinates
void time_operators(const mggen_config& c, const Tree& t, const MeshLevel& m, const LevelOut& L,
                    const std::vector<double>& lumped, TimeOps& T) {
  const int dim = c.dim, nb = 1 << dim, B = c.block;
  const int32_t n = m.n;
  const int64_t N = int64_t(n) * B;
  if (N >= (int64_t(1) << 31)) throw Fail(MGGEN_EINVAL, "too many DoFs for int32 indices");
  T.n_dofs = int32_t(N);
  // Dirichlet DoFs: listed components of nodes on the Dirichlet faces (hanging ones too)
  std::vector<int32_t> gpos(size_t(N), -1);
  for (int32_t i = 0; i < n; ++i) {
    bool on = false;
    for (int a = 0; a < dim; ++a) {
      const int64_t top = t.nc[a] << t.D;
      if ((c.dir_faces >> (2 * a) & 1) && m.lat[3 * i + a] == 0) on = true;
      if ((c.dir_faces >> (2 * a + 1) & 1) && m.lat[3 * i + a] == top) on = true;
    }
    if (!on) continue;
    for (int ci = 0; ci < B; ++ci)
      if (c.dir_comps >> ci & 1) {
        gpos[size_t(i) * B + ci] = int32_t(T.gidx.size());
        T.gidx.push_back(i * B + ci);
      }
  }
  T.n_g = int32_t(T.gidx.size());
  std::vector<std::vector<std::pair<int32_t, double>>> rows;
  rows.resize(size_t(N));
  auto add = [&](int64_t r, int32_t col, double v) {
    for (auto& e : rows[size_t(r)])
      if (e.first == col) { e.second += v; return; }
    rows[size_t(r)].push_back({col, v});
  };
  // Q = Z H^T M_l: node k's mass goes to k, or to the masters of a hanging k
  for (int32_t k = 0; k < n; ++k) {
    const Expand ek = expand(m, k);
    for (int q = 0; q < ek.cnt; ++q)
      for (int ci = 0; ci < B; ++ci) {
        const int64_t r = int64_t(ek.node[q]) * B + ci;
        if (!L.mask[size_t(r)]) add(r, int32_t(int64_t(k) * B + ci), ek.w[q] * lumped[k]);
      }
  }
  // -G = -Z H^T A_full E_g: element couplings of free (expanded) rows with Dirichlet corners
  const double hf = t.hf();
  std::vector<double> krow(size_t(nb) * B * B);
  for (size_t e = 0; e < m.leaves.size(); ++e) {
    bool touches = false;
    for (int b = 0; b < nb && !touches; ++b)
      for (int cj = 0; cj < B; ++cj) touches |= gpos[size_t(m.corner[e * nb + b]) * B + cj] >= 0;
    if (!touches) continue;
    const Leaf& Lf = m.leaves[e];
    const double s = hf * double(Lf.s);
    const double x0[3] = {double(Lf.a[0]) * hf, double(Lf.a[1]) * hf, double(Lf.a[2]) * hf};
    for (int a = 0; a < nb; ++a) {
      const Expand ea = expand(m, m.corner[e * nb + a]);
      element_row(c, a, s, x0, krow.data());
      for (int b = 0; b < nb; ++b) {
        const int32_t jb = m.corner[e * nb + b];
        for (int cj = 0; cj < B; ++cj) {
          const int32_t g = gpos[size_t(jb) * B + cj];
          if (g < 0) continue;
          for (int q = 0; q < ea.cnt; ++q)
            for (int ci = 0; ci < B; ++ci) {
              const int64_t r = int64_t(ea.node[q]) * B + ci;
              if (L.mask[size_t(r)]) continue;
              const double v = ea.w[q] * krow[(size_t(b) * B + ci) * B + cj];
              if (v != 0.0) add(r, int32_t(N + g), -v);
            }
        }
      }
    }
  }
  T.rrow.assign(size_t(N) + 1, 0);
  for (int64_t r = 0; r < N; ++r) {
    std::sort(rows[size_t(r)].begin(), rows[size_t(r)].end());
    T.rrow[size_t(r) + 1] = T.rrow[size_t(r)] + int32_t(rows[size_t(r)].size());
  }
  for (auto& rw : rows)
    for (auto& e : rw) {
      T.rcol.push_back(e.first);
      T.rval.push_back(e.second);
    }
  // H at DoF level
  T.hrow.assign(size_t(N) + 1, 0);
  for (int32_t k = 0; k < n; ++k) {
    Expand ek = expand(m, k);
    std::vector<std::pair<int32_t, double>> ent;
    for (int q = 0; q < ek.cnt; ++q) ent.push_back({ek.node[q], ek.w[q]});
    std::sort(ent.begin(), ent.end());
    for (int ci = 0; ci < B; ++ci) {
      for (auto& pr : ent) {
        T.hcol.push_back(pr.first * B + ci);
        T.hval.push_back(pr.second);
      }
      T.hrow[size_t(k) * B + ci + 1] = int32_t(T.hcol.size());
    }
  }
  T.coords.resize(size_t(n) * dim);
  for (int32_t i = 0; i < n; ++i)
    for (int a = 0; a < dim; ++a) T.coords[size_t(i) * dim + a] = double(m.lat[3 * i + a]) * hf;
}

}  // namespace

struct mggen_problem {
  mggen_config cfg;
  std::vector<LevelOut> levels;
  std::vector<double> rhs;
  TimeOps time;
  bool has_time = false;
  // finest mesh data kept for the noise right-hand side
  std::vector<double> lumped;               // lumped mass per finest node
  std::vector<int32_t> hang_node, hang_master;
  std::vector<double> hang_weight;
  std::vector<uint8_t> mask;
};

extern "C" {

int mggen_build(const mggen_config* cfg, mggen_problem** out) {
  try {
    if (!cfg || !out) throw Fail(MGGEN_EINVAL, "null argument");
    if (cfg->dim != 2 && cfg->dim != 3) throw Fail(MGGEN_EINVAL, "dim must be 2 or 3");
    if (cfg->block < 1 || cfg->block > 8) throw Fail(MGGEN_EINVAL, "block must be 1..8");
    if (cfg->n_rounds < 0 || cfg->n_rounds > 14) throw Fail(MGGEN_EINVAL, "n_rounds out of range");
    for (int a = 0; a < cfg->dim; ++a)
      if (cfg->coarse[a] < 1) throw Fail(MGGEN_EINVAL, "coarse cells must be positive");
    if ((cfg->pde == MGGEN_PDE_ELASTICITY && cfg->block != cfg->dim) ||
        (cfg->pde == MGGEN_PDE_OSEEN && (cfg->block != 4 || cfg->dim != 3)) ||
        ((cfg->pde == MGGEN_PDE_POISSON || cfg->pde == MGGEN_PDE_TD) && cfg->block != 1))
      throw Fail(MGGEN_EINVAL, "block size does not match the pde");
    std::unique_ptr<mggen_problem> P(new mggen_problem());
    P->cfg = *cfg;
    P->cfg.rounds = nullptr;
    Tree t;
    t.init(cfg->dim, cfg->coarse, cfg->h0, cfg->n_rounds);
    for (int r = 0; r < cfg->n_rounds; ++r) apply_round(t, cfg->rounds[r]);
    std::vector<Tree> trees{t};
    while (trees.back().max_leaf_depth() > 0) trees.push_back(coarsen(trees.back()));
    std::reverse(trees.begin(), trees.end());
    const int nl = int(trees.size());
    std::vector<MeshLevel> meshes(nl);
    for (int l = 0; l < nl; ++l) meshes[l] = make_mesh(trees[l]);
    P->levels.resize(nl);
    for (int l = 0; l < nl; ++l) {
      assemble(P->cfg, trees[l], meshes[l], P->levels[l], l == nl - 1 ? &P->rhs : nullptr);
      P->levels[l].max_depth = trees[l].max_leaf_depth();
      if (l > 0) prolongation(trees[l], meshes[l], trees[l - 1], meshes[l - 1], P->levels[l]);
    }
    // lumped mass on the finest mesh: m_i = sum over cells touching i of |K| / 2^d
    const MeshLevel& mf = meshes[nl - 1];
    const int nb = 1 << cfg->dim;
    P->lumped.assign(mf.n, 0.0);
    const double hf = trees[nl - 1].hf();
    for (size_t e = 0; e < mf.leaves.size(); ++e) {
      const double s = hf * double(mf.leaves[e].s);
      const double vol = cfg->dim == 3 ? s * s * s : s * s;
      for (int a = 0; a < nb; ++a) P->lumped[mf.corner[e * nb + a]] += vol / double(nb);
    }
    if (cfg->time_ops) {
      time_operators(P->cfg, trees[nl - 1], mf, P->levels[nl - 1], P->lumped, P->time);
      P->has_time = true;
    }
    P->mask = P->levels[nl - 1].mask;
    P->hang_node = P->levels[nl - 1].hang_node;
    P->hang_master = P->levels[nl - 1].hang_master;
    P->hang_weight = P->levels[nl - 1].hang_weight;
    *out = P.release();
    return MGGEN_OK;
  } catch (const Fail& f) {
    g_err = f.what();
    return f.code;
  } catch (const std::bad_alloc&) {
    g_err = "out of host memory";
    return MGGEN_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return MGGEN_EINTERNAL;
  }
}

int32_t mggen_num_levels(const mggen_problem* p) { return p ? int32_t(p->levels.size()) : 0; }

int mggen_level(const mggen_problem* p, int32_t level, mggen_level_view* o) {
  if (!p || !o || level < 0 || level >= int32_t(p->levels.size())) {
    g_err = "bad level index";
    return MGGEN_EINVAL;
  }
  const LevelOut& L = p->levels[level];
  std::memset(o, 0, sizeof(*o));
  o->n_nodes = L.n;
  o->block = L.block;
  o->nnzb = L.rowptr.empty() ? 0 : L.rowptr.back();
  o->rowptr = L.rowptr.data();
  o->col = L.col.data();
  o->val = L.val.data();
  o->p_cols = L.p_cols;
  o->p_nnz = L.prow.empty() ? 0 : L.prow.back();
  o->p_rowptr = L.prow.empty() ? nullptr : L.prow.data();
  o->p_col = L.pcol.data();
  o->p_val = L.pval.data();
  o->dof_mask = L.mask.data();
  o->n_hanging = int32_t(L.hang_node.size());
  o->hang_node = L.hang_node.data();
  o->hang_master = L.hang_master.data();
  o->hang_weight = L.hang_weight.data();
  o->node_lattice = L.lat.data();
  o->max_depth = L.max_depth;
  return MGGEN_OK;
}

const double* mggen_rhs(const mggen_problem* p) {
  if (!p || p->cfg.rhs == MGGEN_RHS_NOISE) return nullptr;
  return p->rhs.data();
}

int mggen_rhs_noise(const mggen_problem* p, const double* xi, int32_t nrhs, double* out) {
  if (!p || !xi || !out || nrhs < 1 || p->cfg.block != 1) {
    g_err = "mggen_rhs_noise: bad arguments (scalar problems only)";
    return MGGEN_EINVAL;
  }
  const int32_t n = int32_t(p->lumped.size());
  for (int32_t i = 0; i < n; ++i)
    for (int32_t r = 0; r < nrhs; ++r) out[size_t(i) * nrhs + r] = p->lumped[i] * xi[size_t(i) * nrhs + r];
  // H^T: add every hanging value onto its masters, then clear constrained rows
  for (size_t k = 0; k < p->hang_node.size(); ++k) {
    const int32_t h = p->hang_node[k];
    for (int q = 0; q < 4; ++q) {
      const int32_t m = p->hang_master[4 * k + q];
      if (m < 0) continue;
      for (int32_t r = 0; r < nrhs; ++r)
        out[size_t(m) * nrhs + r] += p->hang_weight[4 * k + q] * out[size_t(h) * nrhs + r];
    }
  }
  for (int32_t i = 0; i < n; ++i)
    if (p->mask[i])
      for (int32_t r = 0; r < nrhs; ++r) out[size_t(i) * nrhs + r] = 0.0;
  return MGGEN_OK;
}

int mggen_time_ops(const mggen_problem* p, mggen_time_view* o) {
  if (!p || !o || !p->has_time) {
    g_err = "no time-stepping operators (build with time_ops = 1)";
    return MGGEN_EINVAL;
  }
  const TimeOps& T = p->time;
  std::memset(o, 0, sizeof(*o));
  o->n_dofs = T.n_dofs;
  o->n_g = T.n_g;
  o->r_nnz = int64_t(T.rcol.size());
  o->h_nnz = int64_t(T.hcol.size());
  o->R_rowptr = T.rrow.data();
  o->R_col = T.rcol.data();
  o->R_val = T.rval.data();
  o->H_rowptr = T.hrow.data();
  o->H_col = T.hcol.data();
  o->H_val = T.hval.data();
  o->g_idx = T.gidx.data();
  o->coords = T.coords.data();
  return MGGEN_OK;
}

int mggen_level_cells(const mggen_problem* p, int32_t level, mggen_cells_view* o) {
  if (!p || !o || level < 0 || level >= int32_t(p->levels.size())) {
    g_err = "bad problem, level or output";
    return MGGEN_EINVAL;
  }
  const LevelOut& L = p->levels[size_t(level)];
  o->corners = 1 << p->cfg.dim;
  o->n_cells = int32_t(L.cell_size.size());
  o->corner = L.cells.data();
  o->size = L.cell_size.data();
  return MGGEN_OK;
}

void mggen_free(mggen_problem* p) { delete p; }

const char* mggen_last_error(void) { return g_err.c_str(); }

}  // extern "C"
