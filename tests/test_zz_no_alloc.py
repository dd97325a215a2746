"""fracture_functionals_noalloc (TCV / COD with no allocation: a fixed per-device scratch array)
against fracture_functionals through the C ABI: the same kernels in the same order, so the
values must agree bit for bit, on two calls in a row, the second with a smaller input, and on
batched, adaptive and 3d meshes.  Sizes past the fixed scratch are rejected before device work.
"""
import numpy as np
import pytest

from paper_1806_09924_amd import binding as B
from oracle import mesh as omesh, functionals as ofun
from gpu_util import dev

pytestmark = pytest.mark.gpu


def _fields(xyz, dim, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, (4, dim))
    # a displacement with a nonzero mean and a phase field rising along the last axis, so that
    # TCV and COD are far from zero (no cancellation in the comparisons)
    u = np.stack([1e-3 * (1.0 + 0.5 * np.sin(a[0, k] * xyz[:, 0] + a[1, k] * xyz[:, -1])) for k in range(dim)],
                 axis=1)
    phi = np.clip(0.5 + 0.5 * np.tanh(xyz[:, -1] / 0.3 + 0.2 * a[2, 0] * xyz[:, 0]), 0.0, 1.0)
    return u, phi


def _both(mesh, u, phi, cod_x):
    cod_a, tcv_a = B.functionals(mesh, dev(u), dev(phi), cod_x)
    cod_b, tcv_b = B.functionals(mesh, dev(u), dev(phi), cod_x, noalloc=True)
    return (np.asarray(cod_a), np.asarray(tcv_a)), (np.asarray(cod_b), np.asarray(tcv_b))


def _check_equal(a, b):
    assert np.array_equal(a[0], b[0]), (a[0], b[0])
    assert np.array_equal(a[1], b[1]), (a[1], b[1])


def test_two_calls_second_smaller_uniform_2d():
    L = 2.0
    big = B.Mesh(B.mesh_desc(2, -L, L, 256))
    xyz = big.nodes()[0]
    u, phi = _fields(xyz, 2, 1)
    cod_x = np.array([[-0.3], [-0.1], [0.0], [0.12], [0.5]])
    a, b = _both(big, u, phi, cod_x)
    _check_equal(a, b)
    # anchored to the oracle's functionals on the same fields
    om = omesh.uniform(2, -L, L, 256)
    assert abs(b[1] / ofun.tcv(om, u, phi) - 1.0) <= 1e-12
    oc = np.array([ofun.cod(om, u, phi, x) for x in cod_x])
    assert np.abs(b[0] - oc).max() <= 1e-12 * np.abs(oc).max()
    # a smaller mesh and fewer samples right after: nothing of the larger call may leak in
    small = B.Mesh(B.mesh_desc(2, -1.0, 1.0, 64))
    xs = small.nodes()[0]
    u2, phi2 = _fields(xs, 2, 2)
    a2, b2 = _both(small, u2, phi2, np.array([[0.05], [-0.2]]))
    _check_equal(a2, b2)
    om2 = omesh.uniform(2, -1.0, 1.0, 64)
    assert abs(b2[1] / ofun.tcv(om2, u2, phi2) - 1.0) <= 1e-12
    # TCV only, no COD samples
    _, t3 = B.functionals(small, dev(u2), dev(phi2), noalloc=True)
    assert t3 == b2[1]


def test_batched_adaptive_and_3d():
    descs = [B.mesh_desc(2, -L, L, n) for L, n in ((1.0, 40), (2.5, 96), (0.5, 24))]
    bm = B.Mesh(descs)
    xyz = bm.nodes()[0]
    u, phi = _fields(xyz, 2, 3)
    cod_x = np.array([[[0.0], [0.1]], [[-0.4], [0.2]], [[0.05], [0.0]]])
    a, b = _both(bm, u, phi, cod_x)
    _check_equal(a, b)
    ad = B.Mesh(B.mesh_desc(2, -2.0, 2.0, 16, levels=3, refine_radius=0.3, crack_half_len=0.25))
    assert ad.n_hanging > 0
    u, phi = _fields(ad.nodes()[0], 2, 4)
    a, b = _both(ad, u, phi, np.array([[0.0], [0.1], [0.2]]))
    _check_equal(a, b)
    m3 = B.Mesh(B.mesh_desc(3, -1.0, 1.0, 12))
    u, phi = _fields(m3.nodes()[0], 3, 5)
    a, b = _both(m3, u, phi, np.array([[0.0, 0.0], [0.1, -0.2]]))
    _check_equal(a, b)


def test_rejects_sizes_past_the_scratch():
    m = B.Mesh(B.mesh_desc(2, -1.0, 1.0, 256))
    u, phi = _fields(m.nodes()[0], 2, 6)
    # 256 partial-sum blocks per sample: 3000 samples need about 780k doubles of the 524288
    cod_x = np.zeros((3000, 1))
    with pytest.raises(B.FractureError) as e:
        B.functionals(m, dev(u), dev(phi), cod_x, noalloc=True)
    assert e.value.status == B.FR_EINVAL
    # the allocating entry point takes the same call, and the fixed one still works after it
    cod, tcv = B.functionals(m, dev(u), dev(phi), cod_x[:4])
    cod2, tcv2 = B.functionals(m, dev(u), dev(phi), cod_x[:4], noalloc=True)
    assert np.array_equal(cod, cod2) and tcv == tcv2
