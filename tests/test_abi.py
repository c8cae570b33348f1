"""The C-ABI library: it loads, exports every function include/dbq.h declares, and its host-side
index arithmetic reproduces the oracle's geometry bit for bit (CPU only, no compute calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import wilson as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "dbq.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|char\s*\*|const\s+char\s*\*)\s*\**\s*(\w+)\s*\(",
                       txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["wilson_apply", "gmresdr_first_rhs", "dbicgstab_solve", "project_shifts",
              "link_force", "kappa_critical", "dbq_create", "dbq_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_0710_1988_amd import _abi
    assert os.path.exists(_abi.LIB_PATH), "libdbq.so not built"
    lib = ctypes.CDLL(_abi.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) == set(_abi.EXPORTED)


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4), (6, 4, 2, 10), (8, 12, 4, 6),
                               (20, 20, 20, 32), (24, 24, 24, 48)])
def test_host_geometry_is_bit_exact(L):
    import paper_0710_1988_amd as dbq
    lex, nbr = dbq.geometry_host(L)
    lat = W.Lattice(L, tile=dbq.site_tile(L))
    assert lex.dtype == np.int32
    assert np.array_equal(lex, lat.lex_of_eo)
    k = 0
    for mu in range(4):
        for tab in (lat.fwd[mu], lat.bwd[mu]):
            assert np.array_equal(nbr[k], lat.eo_of_lex[tab[lat.lex_of_eo]])
            k += 1


@pytest.mark.parametrize("L,T", [((24, 24, 24, 48), (4, 4, 4, 4)), ((16, 16, 16, 16), (4, 4, 4, 4)),
                                 ((20, 20, 20, 32), (4, 4, 4, 4)), ((6, 4, 2, 10), (2, 4, 2, 2)),
                                 ((2, 2, 2, 2), (2, 2, 2, 2)), ((12, 6, 4, 8), (4, 2, 4, 4))])
def test_site_tile_rule(L, T):
    """Largest power of two dividing each extent, capped at 4."""
    import paper_0710_1988_amd as dbq
    assert dbq.site_tile(L) == T


def test_host_geometry_rejects_odd_extents():
    from paper_0710_1988_amd import _abi
    lib = _abi.load()
    L = (ctypes.c_int32 * 4)(4, 3, 4, 4)
    buf = (ctypes.c_int32 * 1024)()
    assert lib.dbq_geometry_host(L, buf, buf) == _abi.DBQ_EINVAL


def test_python_binding_rejects_bad_lattices_before_any_call():
    import paper_0710_1988_amd as dbq
    with pytest.raises(ValueError):
        dbq.geometry_host((4, 4, 4, 5))
    with pytest.raises(ValueError):
        dbq.geometry_host((4, 4, 4))


@pytest.mark.parametrize("L", [(24, 24, 24, 48), (16, 16, 16, 16), (20, 20, 20, 32), (8, 8, 8, 8),
                               (4, 4, 4, 4), (6, 4, 2, 10), (12, 12, 12, 12)])
@pytest.mark.parametrize("nch", [1, 3])
def test_tile_schedule_is_a_permutation_with_regions(L, nch):
    """Every LDS-tile launch order visits each (tile, rhs chunk) pair exactly once; order 0 is
    tile-major; orders 1 and 2 keep each of the eight x/y/z half-regions of the tile grid in one
    contiguous run of blocks (one run per XCD when the tile counts are even), and order 2 runs
    the chunks of a region one after the other; order 3 does the same with eight z-half and
    t-quarter regions spanning all of x and y, tile-lexicographic inside, chunks adjacent."""
    import paper_0710_1988_amd as dbq
    T = dbq.site_tile(L)
    NT = [L[i] // T[i] for i in range(4)]
    nt = int(np.prod(NT))
    for order in (0, 1, 2, 3):
        tile, chunk = dbq.tile_schedule_host(L, nch, order)
        pairs = tile.astype(np.int64) * nch + chunk
        assert np.array_equal(np.sort(pairs), np.arange(nt * nch)), order
        if order == 0:
            b = np.arange(nt * nch)
            assert np.array_equal(tile, b // nch) and np.array_equal(chunk, b % nch)
            continue
        if order == 3:
            z = (tile // (NT[0] * NT[1])) % NT[2]
            t = tile // (NT[0] * NT[1] * NT[2])
            zq = (z >= (NT[2] + 1) // 2).astype(int)
            tq = np.array([max(b for b in range(4) if (b * NT[3]) // 4 <= tv) for tv in t])
            region = zq + 2 * tq
            assert np.all(np.diff(region) >= 0)
            for rho in range(8):
                sel = region == rho
                # tiles lexicographic inside the region, the chunks of a tile adjacent
                assert np.all(np.diff(tile[sel][::nch]) > 0)
                assert np.array_equal(chunk[sel], np.tile(np.arange(nch), sel.sum() // nch))
            continue
        tc = [tile % NT[0], (tile // NT[0]) % NT[1], (tile // (NT[0] * NT[1])) % NT[2]]
        half = [(NT[d] + 1) // 2 for d in range(3)]
        region = sum(((tc[d] >= half[d]).astype(int) << d) for d in range(3))
        # regions appear in increasing order, each as one contiguous run
        assert np.all(np.diff(region) >= 0), order
        if all(n % 2 == 0 for n in NT[:3]):
            runs = np.split(region, 8)
            assert all(np.all(r == i) for i, r in enumerate(runs))
        if order == 2:
            for rho in range(8):
                c = chunk[region == rho]
                assert np.all(np.diff(c) >= 0)


def test_tile_schedule_rejects_bad_arguments():
    from paper_0710_1988_amd import _abi
    lib = _abi.load()
    L = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    buf = (ctypes.c_int32 * 16)()
    assert lib.dbq_tile_schedule_host(L, 1, 4, buf, buf) == _abi.DBQ_EINVAL
    assert lib.dbq_tile_schedule_host(L, 0, 1, buf, buf) == _abi.DBQ_EINVAL
