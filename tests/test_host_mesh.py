"""Host logic of libchns (no GPU): the C-ABI library loads, exports every
declared symbol, and its octree build agrees exactly with the oracle's
independently written enumeration (leaves, independent nodes, hanging nodes
and their parents), matched by integer coordinates."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import mesh as om

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "chns.h")).read()
    return sorted(set(re.findall(r"\b(chns_[a-z_]+)\s*\(", txt)) - {"chns_mesh_spec"})


def test_library_exports_every_declared_symbol():
    from paper_2107_05123_amd import _lib
    L = _lib.lib()
    names = _declared_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(_lib.SIGNATURES) <= set(names)
    assert b"gfx950" in L.chns_version()


def _lib_mesh(**kw):
    from paper_2107_05123_amd import Mesh
    return Mesh(**kw)


def _key(coords, side):
    coords = np.asarray(coords, dtype=np.int64)
    k = np.zeros(coords.shape[0], dtype=np.int64)
    for d in range(coords.shape[1] - 1, -1, -1):
        k = k * (side + 1) + coords[:, d]
    return k


def _compare(lib_mesh, orc):
    side = 1 << orc.max_level
    lev, anc = lib_mesh.leaves()
    assert lev.shape[0] == orc.n_elems
    a = sorted(zip(lev.tolist(), _key(anc, side).tolist()))
    b = sorted(zip(orc.level.tolist(), _key(orc.anchor, side).tolist()))
    assert a == b
    lc = lib_mesh.node_coords()
    assert lc.shape[0] == orc.n_indep
    assert np.array_equal(np.sort(_key(lc, side)), np.sort(_key(orc.indep_coords(), side)))
    hc, par = lib_mesh.hanging()
    assert hc.shape[0] == int(orc.hanging.sum())
    # parents as coordinate sets, per hanging node
    lib_par = {}
    for h in range(hc.shape[0]):
        p = par[h][par[h] >= 0]
        lib_par[int(_key(hc[h:h + 1], side)[0])] = sorted(_key(lc[p], side).tolist())
    P = orc.P.tocsr()
    ocoords = orc.indep_coords()
    for n in np.nonzero(orc.hanging)[0]:
        cols = P.indices[P.indptr[n]:P.indptr[n + 1]]
        k = int(_key(orc.nodes[n:n + 1], side)[0])
        assert lib_par[k] == sorted(_key(ocoords[cols], side).tolist())
    info = lib_mesh.summary()
    assert sum(info["elems_in_bricks"]) == orc.n_elems


@pytest.mark.parametrize("dim,level", [(2, 3), (2, 6), (3, 1), (3, 3), (3, 4)])
def test_uniform_matches_oracle(dim, level):
    m = _lib_mesh(dim=dim, min_level=level, max_level=level, rule="uniform")
    _compare(m, om.uniform(dim, level))
    s = m.summary()
    assert s["uniform"] and s["n_hanging"] == 0
    # node order of uniform meshes is lexicographic with x fastest
    c = m.node_coords()
    n1 = (1 << level) + 1
    idx = sum(c[:, d] * n1 ** d for d in range(dim))
    assert np.array_equal(idx, np.arange(c.shape[0]))


@pytest.mark.parametrize("dim,lmin,lmax,band", [(3, 2, 5, 0.03), (3, 1, 6, 0.02), (2, 2, 7, 0.02), (3, 3, 6, 0.05)])
def test_sphere_band_matches_oracle(dim, lmin, lmax, band):
    c = (0.5, 0.3, 0.5)[:dim]
    m = _lib_mesh(dim=dim, min_level=lmin, max_level=lmax, rule="sphere_band", centres=[c], radii=[0.15],
                  band=band)
    orc = om.sphere_band(dim, lmin, lmax, c, 0.15, band)
    assert orc.hanging.any()
    _compare(m, orc)
    assert om.is_balanced(*m.leaves(), lmax) if m.n_elems < 3000 else True


def _blocked_key(c, dim):
    # aligned 8^d blocks of the finest grid in Morton order (bit b of
    # coordinate d at position dim b + d), x fastest inside a block
    c = np.asarray(c, dtype=np.int64)
    blk, low = c >> 3, c & 7
    key = np.zeros(c.shape[0], dtype=np.int64)
    for b in range(20):
        for d in range(dim):
            key |= ((blk[:, d] >> b) & 1) << (dim * b + d)
    inner = sum(low[:, d] << (3 * d) for d in range(dim))
    return (key << (3 * dim)) | inner


@pytest.mark.parametrize("dim,lmax", [(3, 6), (2, 7)])
def test_adaptive_node_order_is_blocked(dim, lmax):
    c = (0.5, 0.3, 0.5)[:dim]
    m = _lib_mesh(dim=dim, min_level=2, max_level=lmax, rule="sphere_band", centres=[c], radii=[0.15], band=0.03)
    assert m.info.node_order == 2 and not m.summary()["uniform"]
    k = _blocked_key(m.node_coords()[:, :dim], dim)
    assert np.all(np.diff(k) > 0)


def test_multi_sphere_and_callback_rules():
    cs = [(0.3, 0.3, 0.3), (0.7, 0.6, 0.5)]
    rs = [0.1, 0.15]
    m = _lib_mesh(dim=3, min_level=2, max_level=5, rule="multi_sphere_band", centres=cs, radii=rs, band=0.03)

    def pred(lev, lo, hi):
        return any(om.box_meets_shell(lo, hi, np.array(c), r - 0.03, r + 0.03) for c, r in zip(cs, rs))

    _compare(m, om.from_predicate(3, 2, 5, pred))

    # callback: refine octants touching the plane x = 1/3 (anchors in units of 2^-max_level)
    L = 6

    def cb(anchor, level):
        s = 1 << (L - level)
        return anchor[0] <= (1 << L) / 3 <= anchor[0] + s

    m2 = _lib_mesh(dim=2, min_level=1, max_level=L, rule="callback", refine=cb)

    def pred2(lev, lo, hi):
        return lo[0] <= 1 / 3 <= hi[0]

    _compare(m2, om.from_predicate(2, 1, L, pred2))


def test_brick_size_heuristic_keeps_enough_bricks():
    # automatic choice: the largest brick edge leaving >= 1024 bricks
    for level, expect in ((7, [4096, 0, 0, 0]), (6, [0, 4096, 0, 0]), (5, [0, 0, 4096, 0]), (3, [0, 0, 0, 512])):
        m = _lib_mesh(dim=3, min_level=level, max_level=level, rule="uniform")
        assert m.summary()["n_bricks"] == expect, level


def test_bricks_cover_uniform_mesh_with_largest_bricks():
    m = _lib_mesh(dim=3, min_level=5, max_level=5, rule="uniform", brick_max=8)
    s = m.summary()
    assert s["n_bricks"] == [64, 0, 0, 0]
    assert s["n_colors"] == 8
    # shared nodes: every node on a brick face (multiples of 8 in some coordinate)
    c = m.node_coords()
    on_face = np.any(c % 8 == 0, axis=1)
    assert s["n_shared"] == int(on_face.sum())


def test_bad_specs_are_rejected():
    from paper_2107_05123_amd import ChnsError
    with pytest.raises(ChnsError):
        _lib_mesh(dim=4, min_level=1, max_level=2)
    with pytest.raises(ChnsError):
        _lib_mesh(dim=3, min_level=3, max_level=2)
    with pytest.raises(ChnsError):
        _lib_mesh(dim=3, min_level=1, max_level=3, rule="sphere_band")


def test_threaded_host_build_is_repeatable():
    """The octree, node and table builds split work over the host threads
    (lock-free hash-set fills, per-chunk passes merged in chunk order):
    building, remeshing and the transfer twice give identical results."""
    from paper_2107_05123_amd import Transfer
    spec = dict(dim=3, min_level=3, max_level=8, rule="sphere_band", centres=[(0.5, 0.3, 0.5)], radii=[0.15],
                band=0.03)
    a, b = _lib_mesh(**spec), _lib_mesh(**spec)
    assert a.n_elems > 8 * (1 << 14)  # enough leaves for every thread to take a chunk
    for f in (lambda m: m.leaves(), lambda m: (m.node_coords(),), lambda m: m.hanging()):
        for x, y in zip(f(a), f(b)):
            assert np.array_equal(x, y)
    assert a.summary() == b.summary()
    c = a.node_coords() / float(1 << 8)
    phi = np.tanh((0.15 - np.linalg.norm(c - np.array([0.5, 0.32, 0.5]), axis=1)) / 0.02)
    ra, rb = a.remesh(phi, 3, threshold=0.9), b.remesh(phi, 3, threshold=0.9)
    assert np.array_equal(ra.node_coords(), rb.node_coords()) and ra.summary() == rb.summary()
    ta, tb = Transfer(a, ra).matrix(), Transfer(b, rb).matrix()
    for x, y in zip(ta, tb):
        assert np.array_equal(x, y)
