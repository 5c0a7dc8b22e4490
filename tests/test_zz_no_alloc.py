"""The allocation-free outer defect (mg_outer_defect_noalloc) against mg_outer_defect,
through the C ABI: same residual and norm, on two calls in a row that share the static
scratch array, the second on a smaller problem, and the refusal of finest levels whose
partial sums do not fit the array."""
import ctypes as C
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


def _handle(wl):
    from paper_2405_05047_amd import gen, mg
    p = gen.build(wl)
    return p, mg.Hierarchy(p.levels, mg.config_from(wl))


def _both(h, N, seed):
    b = torch.from_numpy(W.rand_vec(seed, N)).cuda()
    x = torch.from_numpy(W.rand_vec(seed + 1, N)).cuda()
    r_ref = torch.empty_like(b)
    n_ref = torch.zeros(1, dtype=torch.float64, device="cuda")
    h.outer_defect(b, x, r_ref, n_ref)
    r = torch.full_like(b, np.nan)
    n = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    h.outer_defect_noalloc(b, x, r, n)
    torch.cuda.synchronize()
    return r_ref.cpu().numpy(), n_ref.cpu().numpy(), r.cpu().numpy(), n.cpu().numpy(), b.cpu().numpy(), x.cpu().numpy()


def test_noalloc_defect_matches_the_allocating_entry_point():
    """Two calls in a row (larger problem, then a smaller one): both equal mg_outer_defect
    bit for bit (same kernels, same partial-sum order); the residual also matches a host
    CSR product to 1e-12 of |A||x| + |b|."""
    import scipy.sparse as sp
    for wl in (W.c2_td(band_rounds=3, uniform_rounds=1), W.c1_poisson(4)):
        p, h = _handle(wl)
        top = p.finest
        N = top.n * top.block
        _log(wl.name, N, "DoFs")
        r_ref, n_ref, r, n, b, x = _both(h, N, 11)
        assert np.array_equal(r, r_ref) and np.array_equal(n, n_ref), wl.name
        A = sp.bsr_matrix((top.val, top.col, top.rowptr), shape=(N, N)).tocsr()
        scale = (abs(A) @ np.abs(x) + np.abs(b)).max()
        assert np.abs(r - (b - A @ x)).max() <= 1e-12 * scale
        assert abs(n[0] - np.linalg.norm(b - A @ x)) <= 1e-12 * np.linalg.norm(b - A @ x)


def test_noalloc_refuses_levels_beyond_the_array():
    """With the array's usable size lowered below the finest level's partial count
    (test-only MGQ1_SCRATCH_LIMIT, read at setup) the call is refused before device work
    and leaves its outputs untouched; run in a child process so the setting stays there."""
    code = r'''
import numpy as np, torch, workloads as W
from paper_2405_05047_amd import gen, mg
wl = W.c2_td(band_rounds=3, uniform_rounds=1)
p = gen.build(wl)
h = mg.Hierarchy(p.levels, mg.config_from(wl))
N = p.finest.n
b = torch.ones(N, dtype=torch.float64, device="cuda")
x = torch.zeros_like(b)
r = torch.full_like(b, 7.0)
nrm = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
try:
    h.outer_defect_noalloc(b, x, r, nrm)
    print("NOT REFUSED")
except mg.MGError as e:
    torch.cuda.synchronize()
    assert e.code == -7 and "partial sums" in str(e), e
    assert bool((r == 7.0).all()) and float(nrm[0]) == 7.0
    print("REFUSED OK")
'''
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, MGQ1_SCRATCH_LIMIT="1", PYTHONPATH=root)
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True,
                         timeout=120)
    _log(out.stdout.strip(), out.stderr.strip()[-300:])
    assert out.returncode == 0 and "REFUSED OK" in out.stdout
