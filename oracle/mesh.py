"""Adaptive quadrilateral / hexahedral meshes with hanging nodes (oracle, test-only).

Follows Sec. 2.2 of the paper ("Adaptivity and geometric multigrid hierarchy"):
a refined cell is replaced by 2^d children, neighbouring cells differ by at most one
level, nodes on edges/faces of a coarser neighbour are hanging nodes that are replaced
by interpolation of their neighbours through a square sparse matrix H (identity on
regular rows, interpolation weights on hanging rows), and the multigrid hierarchy is
built by global coarsening that takes back as many refinements as possible, a family
being coarsened when all of its 2^d children are leaves (Fig. "fig:coarsening").

Representation (chosen to be obviously correct rather than fast): every leaf is stored
implicitly through a depth map over the finest cell lattice -- each finest lattice cell
holds the depth of the leaf that covers it.  Depth 0 is a coarse-grid cell.  Lattice
arrays are indexed (z, y, x) (2D: (y, x)), so C-order flattening is the lexicographic
(z, y, x) ordering used for node numbers.

Readings of the paper (its text leaves these open):
  * "level jump of 1 for neighboring elements" is read over shared vertices: no leaf may
    share a vertex with a leaf two or more levels deeper.  This keeps every master of a
    hanging node regular, so one application of H is enough (H^2 = H).
  * In 3D both edge midpoints (2 masters, weight 1/2) and face centres (4 masters,
    weight 1/4) are hanging nodes.
  * Global coarsening step: candidate families are those whose children are all leaves;
    candidates whose coarsened father would share a vertex with a staying leaf two or
    more levels deeper are dropped until nothing changes; the rest are coarsened
    together.  This is the largest admissible set, so it does not depend on any order.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def _upsample(m: np.ndarray, f: int) -> np.ndarray:
    """Repeat every entry of `m` f times along each axis."""
    for ax in range(m.ndim):
        m = np.repeat(m, f, axis=ax)
    return m


def _block_reduce(a: np.ndarray, f: int, fn) -> np.ndarray:
    """Reduce non-overlapping f^dim blocks of `a` with numpy reduction `fn`."""
    shp = []
    for n in a.shape:
        shp += [n // f, f]
    r = a.reshape(shp)
    return fn(r, axis=tuple(range(1, 2 * a.ndim, 2)))


def _neighbour_max(dep: np.ndarray) -> np.ndarray:
    """Largest depth among the 3^dim finest cells that share a vertex with each cell."""
    pad = np.pad(dep.astype(np.int16), 1, constant_values=-1)
    out = np.full(dep.shape, -1, np.int16)
    for off in itertools.product((0, 1, 2), repeat=dep.ndim):
        sl = tuple(slice(o, o + n) for o, n in zip(off, dep.shape))
        np.maximum(out, pad[sl], out=out)
    return out


class Forest:
    """A forest of quadtrees (dim=2) or octrees (dim=3) over a box of coarse cells."""

    def __init__(self, dim: int, coarse, h0: float, max_depth: int):
        self.dim = dim
        self.coarse = tuple(int(c) for c in coarse)          # (x, y[, z])
        self.h0 = float(h0)
        self.D = int(max_depth)
        self.cell_shape = tuple(c << self.D for c in reversed(self.coarse))  # (z,) y, x
        self.dep = np.zeros(self.cell_shape, np.int8)

    def copy(self) -> "Forest":
        f = Forest(self.dim, self.coarse, self.h0, self.D)
        f.dep = self.dep.copy()
        return f

    # ------------------------------------------------------------------ geometry
    @property
    def vshape(self):
        return tuple(n + 1 for n in self.cell_shape)

    @property
    def hf(self) -> float:
        """Edge length of one finest lattice cell."""
        return self.h0 / (1 << self.D)

    def max_depth(self) -> int:
        return int(self.dep.max())

    def depths(self):
        return [int(d) for d in np.unique(self.dep)]

    def leaf_grid(self, d: int) -> np.ndarray:
        """Boolean array over the depth-d cell grid: True where a depth-d leaf sits.

        The finest cell at the lower corner of a depth-d grid cell has depth d exactly
        when that grid cell is itself a leaf."""
        s = 1 << (self.D - d)
        return self.dep[(slice(None, None, s),) * self.dim] == d

    def leaves(self):
        """All leaves as (depth (n,), lower-corner lattice coords (n, dim) ordered (x, y[, z]))."""
        ds, anc = [], []
        for d in self.depths():
            s = 1 << (self.D - d)
            idx = np.nonzero(self.leaf_grid(d))
            a = np.stack([idx[k] * s for k in reversed(range(self.dim))], axis=1)
            ds.append(np.full(len(a), d, np.int64))
            anc.append(a.astype(np.int64))
        return np.concatenate(ds), np.concatenate(anc)

    # ------------------------------------------------------------------ refinement
    def refine_marked(self, marks: dict) -> None:
        """Replace every marked leaf by its 2^dim children (Sec. 2.2).

        `marks[d]` is a boolean array over the depth-d grid (only entries that are
        depth-d leaves are honoured)."""
        add = np.zeros(self.cell_shape, bool)
        for d, m in marks.items():
            if d >= self.D:
                if np.any(m & self.leaf_grid(d)):
                    raise ValueError("refinement beyond the lattice depth")
                continue
            m = m & self.leaf_grid(d)
            if m.any():
                add |= _upsample(m, 1 << (self.D - d))
        self.dep[add] += 1

    def is_balanced(self) -> bool:
        return not np.any(_neighbour_max(self.dep) >= self.dep.astype(np.int16) + 2)

    def balance(self) -> int:
        """Refine leaves until no leaf shares a vertex with a leaf two or more levels
        deeper (reading of the one-level-jump rule of Sec. 2.2).  Returns #rounds."""
        it = 0
        while True:
            need = _neighbour_max(self.dep) >= self.dep.astype(np.int16) + 2
            if not need.any():
                return it
            marks = {}
            for d in self.depths():
                f = 1 << (self.D - d)
                marks[d] = _block_reduce(need & (self.dep == d), f, np.any)
            self.refine_marked(marks)
            it += 1

    def apply_round(self, rule: tuple) -> None:
        """One refinement round of a workload recipe, followed by balancing."""
        kind = rule[0]
        marks = {}
        dmax = self.max_depth()
        for d in self.depths():
            g = self.leaf_grid(d)
            if kind == "uniform":
                marks[d] = g
                continue
            s = 1 << (self.D - d)
            idx = np.indices(g.shape)                      # (z,) y, x grid indices
            lo = [idx[self.dim - 1 - a] * s for a in range(self.dim)]   # per axis a (x, y, z)
            if kind == "band":
                _, cx, cy, r, delta = rule
                hf = self.hf
                x0 = lo[0] * hf
                y0 = lo[1] * hf
                x1 = (lo[0] + s) * hf
                y1 = (lo[1] + s) * hf
                # nearest and farthest point of the closed box from the centre
                nx = np.clip(cx, x0, x1) - cx
                ny = np.clip(cy, y0, y1) - cy
                dmin2 = nx * nx + ny * ny
                fx = np.maximum(np.abs(x0 - cx), np.abs(x1 - cx))
                fy = np.maximum(np.abs(y0 - cy), np.abs(y1 - cy))
                dmax2 = fx * fx + fy * fy
                ro = r + delta
                ri = r - delta
                hit = (dmin2 < ro * ro) & (dmax2 > ri * ri) if ri > 0 else (dmin2 < ro * ro)
                marks[d] = g & hit
            elif kind == "corner":
                _, axes, thr = rule
                if d != dmax:
                    continue
                ok = np.ones(g.shape, bool)
                for a in range(self.dim):
                    if axes >> a & 1:
                        ok &= (lo[a] + s) * self.hf <= thr
                marks[d] = g & ok
            else:
                raise ValueError(f"unknown refinement rule {kind}")
        self.refine_marked(marks)
        self.balance()

    # ------------------------------------------------------------------ coarsening
    def coarsened(self) -> "Forest":
        """One global coarsening step (Sec. 2.2, Fig. "fig:coarsening")."""
        dep = self.dep
        cand = np.zeros(self.cell_shape, bool)
        for d in range(1, self.max_depth() + 1):
            f = 1 << (self.D - d + 1)          # size of the father cell in lattice units
            bmin = _block_reduce(dep, f, np.min)
            bmax = _block_reduce(dep, f, np.max)
            cand |= _upsample((bmin == d) & (bmax == d), f)
        while True:
            new = dep - cand.astype(np.int8)
            viol = _neighbour_max(new) >= new.astype(np.int16) + 2
            if not viol.any():
                break
            assert not np.any(viol & ~cand)
            for d in range(1, self.max_depth() + 1):
                f = 1 << (self.D - d + 1)
                drop = _block_reduce(viol & cand & (dep == d), f, np.any)
                cand &= ~_upsample(drop, f)
        out = self.copy()
        out.dep = (dep - cand.astype(np.int8)).astype(np.int8)
        return out

    # ------------------------------------------------------------------ nodes
    def node_mask(self) -> np.ndarray:
        """Vertex-lattice mask of mesh nodes: lattice points that are a corner of a leaf."""
        V = np.zeros(self.vshape, bool)
        for d in self.depths():
            g = self.leaf_grid(d)
            s = 1 << (self.D - d)
            C = np.zeros(tuple(n + 1 for n in g.shape), bool)
            for off in itertools.product((0, 1), repeat=self.dim):
                sl = tuple(slice(o, o + n) for o, n in zip(off, g.shape))
                C[sl] |= g
            V[(slice(None, None, s),) * self.dim] |= C
        return V

    def hanging(self, V: np.ndarray):
        """Hanging nodes and their masters (Sec. 2.2).

        A node is hanging when it lies inside an edge or a face of some leaf.  Under the
        2:1 rule it is the midpoint of that edge (masters: the edge ends, 1/2 each) or the
        centre of that face (masters: the 4 face corners, 1/4 each).
        Returns (lattice index of the hanging points (k,), masters (k, 4), weights (k, 4),
        number of masters per point (k,)), in lattice linear indices, unused slots -1 / 0.
        """
        vs = self.vshape
        pts, mas, wts, cnt = [], [], [], []

        def lin(p):                              # p: (n, dim) in (x, y[, z]) order
            return np.ravel_multi_index(tuple(p[:, a] for a in reversed(range(self.dim))), vs)

        for d in self.depths():
            s = 1 << (self.D - d)
            if s < 2:
                continue
            h = s // 2
            idx = np.nonzero(self.leaf_grid(d))
            A = np.stack([idx[k] * s for k in reversed(range(self.dim))], axis=1)
            eye = np.eye(self.dim, dtype=np.int64)
            # edges: along axis a, offset 0 or s in every other axis
            for a in range(self.dim):
                others = [b for b in range(self.dim) if b != a]
                for offs in itertools.product((0, s), repeat=len(others)):
                    shift = sum(o * eye[b] for o, b in zip(offs, others))
                    m = A + shift + h * eye[a]
                    p0 = m - h * eye[a]
                    p1 = m + h * eye[a]
                    ml = lin(m)
                    hit = V.ravel()[ml]
                    if hit.any():
                        k = int(hit.sum())
                        pts.append(ml[hit])
                        mm = np.full((k, 4), -1, np.int64)
                        ww = np.zeros((k, 4))
                        mm[:, 0] = lin(p0[hit])
                        mm[:, 1] = lin(p1[hit])
                        ww[:, :2] = 0.5
                        mas.append(mm)
                        wts.append(ww)
                        cnt.append(np.full(k, 2))
            if self.dim == 3:
                # faces: normal axis n, offset 0 or s along n, centre in the two tangent axes
                for n in range(3):
                    t = [b for b in range(3) if b != n]
                    for o in (0, s):
                        c = A + o * eye[n] + h * eye[t[0]] + h * eye[t[1]]
                        cl = lin(c)
                        hit = V.ravel()[cl]
                        if hit.any():
                            k = int(hit.sum())
                            pts.append(cl[hit])
                            mm = np.full((k, 4), -1, np.int64)
                            for q, (u, v) in enumerate(itertools.product((-h, h), repeat=2)):
                                mm[:, q] = lin(c[hit] + u * eye[t[0]] + v * eye[t[1]])
                            ww = np.full((k, 4), 0.25)
                            mas.append(mm)
                            wts.append(ww)
                            cnt.append(np.full(k, 4))
        if not pts:
            z = np.zeros(0, np.int64)
            return z, np.zeros((0, 4), np.int64), np.zeros((0, 4)), z
        pts = np.concatenate(pts)
        mas = np.concatenate(mas)
        wts = np.concatenate(wts)
        cnt = np.concatenate(cnt)
        u, first = np.unique(pts, return_index=True)
        # every leaf that sees the same hanging point must name the same masters
        order = np.argsort(pts, kind="stable")
        sp_pts = pts[order]
        sp_mas = np.sort(mas[order], axis=1)
        grp = np.searchsorted(u, sp_pts)
        ref = np.sort(mas[first], axis=1)[grp]
        if not np.array_equal(sp_mas, ref):
            raise AssertionError("inconsistent masters for a hanging node")
        return u, mas[first], wts[first], cnt[first]


class Mesh:
    """Nodes, hanging nodes and the hanging-node matrix H of one forest."""

    def __init__(self, forest: Forest):
        self.forest = forest
        self.dim = forest.dim
        V = forest.node_mask()
        self.vmask = V
        flat = V.ravel()
        self.node_lin = np.nonzero(flat)[0]                 # lattice index of node i
        self.n = len(self.node_lin)
        self.node_of_lin = np.full(flat.size, -1, np.int64)
        self.node_of_lin[self.node_lin] = np.arange(self.n)
        zyx = np.unravel_index(self.node_lin, V.shape)
        self.coords_lat = np.stack([zyx[k] for k in reversed(range(self.dim))], axis=1)  # (x,y,z)
        self.coords = self.coords_lat * forest.hf
        hp, hm, hw, hc = forest.hanging(V)
        self.hang_nodes = self.node_of_lin[hp]
        masters = np.where(hm >= 0, self.node_of_lin[np.maximum(hm, 0)], -1)
        if np.any((hm >= 0) & (masters < 0)):
            raise AssertionError("a master of a hanging node is not a mesh node")
        self.hang_masters = masters
        self.hang_weights = hw
        self.hang_count = hc
        self.is_hanging = np.zeros(self.n, bool)
        self.is_hanging[self.hang_nodes] = True
        if np.any(self.is_hanging[masters[masters >= 0]]):
            raise AssertionError("a master of a hanging node is itself hanging")
        self.H = self._build_H()

    def _build_H(self) -> sp.csr_matrix:
        """Square hanging-node matrix (Sec. 2.2): identity rows for regular nodes,
        interpolation weights on the rows of hanging nodes."""
        reg = np.nonzero(~self.is_hanging)[0]
        rows = [reg]
        cols = [reg]
        vals = [np.ones(len(reg))]
        ok = self.hang_masters >= 0
        rows.append(np.repeat(self.hang_nodes, ok.sum(axis=1)))
        cols.append(self.hang_masters[ok])
        vals.append(self.hang_weights[ok])
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.n, self.n))

    def boundary_mask(self, faces: int) -> np.ndarray:
        """Nodes on the selected faces (bit 2a: x_a = 0, bit 2a+1: x_a = max)."""
        on = np.zeros(self.n, bool)
        for a in range(self.dim):
            top = self.forest.cell_shape[self.dim - 1 - a]
            if faces >> (2 * a) & 1:
                on |= self.coords_lat[:, a] == 0
            if faces >> (2 * a + 1) & 1:
                on |= self.coords_lat[:, a] == top
        return on


def build_forest(wl) -> Forest:
    """Coarse grid of `wl`, then its refinement rounds (each followed by balancing)."""
    f = Forest(wl.dim, wl.coarse, wl.h0, max(wl.n_rounds, 0))
    for rule in wl.rounds:
        f.apply_round(rule)
    return f


def hierarchy_forests(finest: Forest):
    """Global coarsening down to the coarse grid; returns [coarsest, ..., finest]."""
    out = [finest]
    while out[-1].max_depth() > 0:
        out.append(out[-1].coarsened())
    return out[::-1]
