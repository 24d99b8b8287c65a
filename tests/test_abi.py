"""C-ABI library: loads, exports every declared symbol, host-side entry points.

No GPU work here: only the host half of the library (patterns, SNF, kernel and
stiffness validation) is called.
"""
import os
import re

import numpy as np
import pytest

from oracle.lattice import Pattern as OPattern
import lsh_inputs as li

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lsh_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol(lib):
    import ctypes
    so = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(so, n)]
    assert declared_symbols(), "no declarations found"
    assert not missing, missing


@pytest.mark.parametrize("M", [
    [[16, 0, 0], [0, 16, 0], [0, 0, 16]],
    [[128, 32, 0], [0, 128, 0], [0, 0, 64]],
    [[8, 2, 0], [0, 8, 0], [0, 0, 4]],
    [[4, 1, 0], [0, 4, 0], [0, 0, 2]],
    [[3, 1, 0], [-1, 2, 1], [0, 1, 4]],
    [[-2, 1, 1], [1, -3, 0], [0, 2, 5]],
    [[5, 0, 0], [0, 5, 0], [0, 0, 7]],
    [[6, -3, 2], [1, 4, 0], [2, 0, 3]],
])
def test_pattern_matches_oracle(lib, M):
    """SNF diagonal equal; same point set exactly; U diag(e) V == M."""
    P = lib.Pattern(M)
    O = OPattern(M)
    assert list(P.e) == list(O.e)
    assert P.m == O.m
    U, V = P.snf()
    np.testing.assert_array_equal(U @ np.diag(P.e) @ V, np.array(M))
    assert abs(round(np.linalg.det(U))) == 1 and abs(round(np.linalg.det(V))) == 1
    if P.m <= 300000:
        a = sorted(map(tuple, P.point_numerators().tolist()))
        b = sorted(map(tuple, O.point_numerators().tolist()))
        assert a == b


def test_pattern_point_map_is_snf_map(lib):
    """y(a) = M^{-1} U a mod 1 in storage order, with the library's own U."""
    M = np.array([[6, -3, 2], [1, 4, 0], [2, 0, 3]])
    P = lib.Pattern(M)
    U, _ = P.snf()
    a = np.array(np.meshgrid(*[np.arange(k) for k in P.e], indexing="ij")).reshape(3, -1).T
    y = (np.linalg.inv(M) @ U @ a.T).T
    y = y - np.floor(y + 0.5)
    np.testing.assert_allclose(P.points(), y, atol=1e-12)


def test_errors_host_side(lib):
    with pytest.raises(lib.LshError) as e:
        lib.Pattern([[2, 4, 0], [1, 2, 0], [0, 0, 1]])
    assert e.value.status == -2  # LSH_ESINGULAR
    P = lib.Pattern(np.diag([4, 4, 4]))
    with pytest.raises(lib.LshError) as e:
        P.set_kernel("dlvp", {"alpha": [0.5, 1.5, 0.5]})
    assert e.value.status == -1
    with pytest.raises(lib.LshError) as e:
        P.set_kernel("box", {"Xi": np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 1.0]])})
    assert e.value.status == -1  # directions do not span R^3
    C = li.isotropic_voigt(1.0, 0.3)
    bad = C.copy()
    bad[0, 0] = -1.0
    with pytest.raises(lib.LshError) as e:
        P.set_stiffness(np.stack([C, bad]), C, np.zeros(64, np.uint8))
    assert e.value.status == -4  # LSH_ENOTELLIPTIC
    nan = C.copy()
    nan[1, 2] = np.nan
    with pytest.raises(lib.LshError) as e:
        P.set_stiffness(np.stack([C, nan]), C, np.zeros(64, np.uint8))
    assert e.value.status == -1
    with pytest.raises(lib.LshError) as e:
        P.set_stiffness(np.stack([C]), C, np.full(64, 3, np.uint8))
    assert e.value.status == -1  # phase index out of range
    with pytest.raises(lib.LshError) as e:
        P.workspace_bytes(2, "fp64") if False else lib._check(lib._lib.lsh_solve_bytes(P._h, 0, 0, None))
    assert e.value.status == -1


def test_unsupported_prime_factor_reported(lib):
    """A prime SNF factor above 13 is refused with LSH_EUNSUPPORTED (host check)."""
    P = lib.Pattern(np.diag([1, 1, 17]))
    with pytest.raises(lib.LshError) as e:
        P.workspace_bytes(1, "fp64")
    assert e.value.status == -9


def test_workspace_sizes_scale(lib):
    P = lib.Pattern(np.diag([16, 16, 16]))
    P.set_kernel("dirichlet")
    b1 = P.workspace_bytes(1, "fp64")
    b6 = P.workspace_bytes(6, "fp64")
    f1 = P.workspace_bytes(1, "fp32")
    assert b6 > 5 * b1 * 0.9 and f1 < b1


def test_unet_host_side(lib):
    """U-Net network description and size queries (host only) agree with the
    reference network's layer table; misuse is reported, not run."""
    import ctypes
    from oracle import unet
    assert lib.UNet.layers() == unet.LAYERS
    so = lib._lib
    h = ctypes.c_void_p()
    assert so.lsh_unet_create(16, ctypes.byref(h)) == -1
    assert so.lsh_unet_create(32, ctypes.byref(h)) == 0
    try:
        cnt = ctypes.c_int64()
        assert so.lsh_unet_param_count(h, ctypes.byref(cnt)) == 0
        assert cnt.value == unet.param_layout()[2]
        nb = ctypes.c_size_t()
        assert so.lsh_unet_act_bytes(h, 12, 1, ctypes.byref(nb)) == -1
        assert so.lsh_unet_act_bytes(h, 16, 1, ctypes.byref(nb)) == 0
        train16 = nb.value
        assert so.lsh_unet_act_bytes(h, 16, 0, ctypes.byref(nb)) == 0
        assert 0 < nb.value < train16
        assert so.lsh_unet_act_bytes(h, 32, 1, ctypes.byref(nb)) == 0
        assert 7.5 * train16 < nb.value < 8.5 * train16
        loss = ctypes.c_double()
        # not bound: rejected before any device work
        assert so.lsh_unet_train_step(h, None, None, 16, 0.0, None, 0, None, ctypes.byref(loss)) == -1
        assert so.lsh_unet_get_params(h, (ctypes.c_float * 1)(), None) == -10
    finally:
        so.lsh_unet_destroy(h)


@pytest.mark.parametrize("M", [[[128, 0], [0, 128]], [[64, 64], [-64, 64]], [[128, 272], [0, 128]],
                               [[5, 2], [1, 4]], [[-3, 1], [2, 6]]])
def test_plane_pattern_matches_oracle(lib, M):
    """d = 2 (Sec. 4's M1, M2, M3 and ragged ones): the library holds
    blockdiag(M, 1) (SNF e1 = 1, U diag(e) V of that), and its 2-D point set is
    the oracle's exactly."""
    P = lib.Pattern(M)
    O = OPattern(M)
    assert P.d == 2 and P.nc == 3 and P.m == O.m
    assert P.e[0] == 1 and list(P.e[1:]) == list(O.e)
    U, V = P.snf()
    M3 = np.zeros((3, 3), dtype=np.int64)
    M3[:2, :2] = M
    M3[2, 2] = 1
    np.testing.assert_array_equal(U @ np.diag(P.e) @ V, M3)
    y = P.point_numerators()
    assert y.shape == (P.m, 2)
    assert sorted(map(tuple, y.tolist())) == sorted(map(tuple, O.point_numerators().tolist()))


def test_plane_errors_host_side(lib):
    P = lib.Pattern([[8, 8], [-8, 8]])
    with pytest.raises(lib.LshError) as e:
        P.set_kernel("dlvp", {"alpha": [0.5, 0.5, 0.5]})     # alpha[d], d = 2
    assert e.value.status == -1
    with pytest.raises(lib.LshError) as e:
        P.set_kernel("box", {"Xi": np.array([[1.0, 2.0, -1.0], [2.0, 4.0, -2.0]]), "R": 2})
    assert e.value.status == -1                              # directions do not span R^2
    P.set_kernel("box", {"Xi": np.array([[1, 0, 1, 0, 1, 0, 1, 0], [0, 1, 0, 1, 0, 1, 0, 1]], float), "R": 16})
    P.set_kernel("dlvp", {"alpha": [0.9, 0.0]})
    C = np.stack([li.isotropic_voigt_plane(1.0, 0.3), li.isotropic_voigt_plane(10.0, 0.3)])
    C0 = li.mean_reference(C)
    P.set_stiffness(C, C0, np.zeros(P.m, np.uint8))
    bad = C.copy()
    bad[1, 2, 2] = -0.5                                      # negative shear modulus
    with pytest.raises(lib.LshError) as e:
        P.set_stiffness(bad, C0, np.zeros(P.m, np.uint8))
    assert e.value.status == -4
    asym = C.copy()
    asym[0, 0, 1] += 0.1
    with pytest.raises(lib.LshError) as e:
        P.set_stiffness(asym, C0, np.zeros(P.m, np.uint8))
    assert e.value.status == -4
    with pytest.raises(lib.LshError) as e:
        lib.Pattern(np.diag([4, 4, 4, 4]))                   # d = 4
    assert e.value.status == -1


def test_box_tail_and_scheme_arguments(lib):
    """The Box tail flag must be 0 or 1; unknown schemes are refused."""
    import ctypes
    P = lib.Pattern(np.diag([4, 4, 4]))
    Xi = [1, 0, 0, 1, 0, 1, 0, 1, 0, 0, 1, 0]                 # 3 x 4, row-major
    for flag, ok in ((0.0, True), (1.0, True), (2.0, False), (0.5, False)):
        arr = np.array([4.0] + [float(v) for v in Xi] + [8.0, flag])
        rc = lib._lib.lsh_set_kernel(P._h, 3, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(arr))
        assert (rc == 0) == ok, (flag, rc)
    P.set_kernel("box", {"Xi": np.array(Xi, float).reshape(3, 4), "R": 8, "tail": True})
    with pytest.raises(lib.LshError) as e:
        lib._check(lib._lib.lsh_set_scheme(P._h, 7))
    assert e.value.status == -1
    for sc in ("ls", "ve", "cg", "ls_inc"):
        P.set_scheme(sc)
    for bad in (-1, 4):
        with pytest.raises(lib.LshError):
            lib._check(lib._lib.lsh_set_scheme(P._h, bad))
