"""GPU parity of every GEMM tile configuration the library carries, forced
with the flow option tile=<bm>x<bk> (the autotuner otherwise picks one per
order), against the FP64 oracle.

n = 500 is padded to 512 inside the library: 2 x 2 output tiles of 256, 4 x 4
of 128 and 8 x 8 of 64, with 8 to 32 K tiles and a ragged tail, so every
kernel runs its K-loop pipeline, its boundary handling and its fused
epilogues (affine and RK4 stage update for the fine propagator, Euler update
for the coarse one) on several tiles."""

import pytest

from oracle import MatrixAlgebra, HOMOTOPY, INV_LINEAR, integrators
from paper_1505_07959_amd import inputs
from tests.gpu_util import dev, host, empty, rel, say

pytestmark = pytest.mark.gpu

# (bm, bk) per dtype, as compiled into the library
TILES = {
    "f64": [(128, 16), (128, 32), (64, 16), (64, 32)],
    "f32": [(128, 32), (128, 16), (64, 32)],
    "bf16": [(128, 64), (128, 32), (256, 32), (256, 64), (64, 64)],
    "f16": [(128, 64), (128, 32), (256, 32), (256, 64), (64, 64)],
    "bf16x3": [(128, 64), (256, 32), (64, 64)],
}
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2, "f16": 1e-2, "bf16x3": 1e-4}
CASES = [(d, bm, bk) for d, ts in TILES.items() for bm, bk in ts]
N = 500


def _check_forced(capfd, bm, bk):
    """the library reports the forced tile for the flow's dtype (verbose=1)"""
    err = capfd.readouterr().err
    assert ("-> bm=%d bk=%d (forced)" % (bm, bk)) in err, err[-400:]


def _case(seed):
    A, _, _ = inputs.spd(N, "uniform", 0.3, 2.0, seed)
    X0 = inputs.perturbed_identity(N, seed + 100, eps=0.1)
    return A, X0


@pytest.mark.parametrize("kind", [HOMOTOPY, INV_LINEAR])
@pytest.mark.parametrize("dtype,bm,bk", CASES)
def test_fine_propagate_every_tile(dtype, bm, bk, kind, capfd):
    from paper_1505_07959_amd import fm
    say("tile %dx%d dtype=%s kind=%d n=%d fine" % (bm, bk, dtype, kind, N))
    A, X0 = _case(11)
    t0, t1, steps = 0.1, 0.3, 4
    ref = integrators.fine(MatrixAlgebra(N), kind, A, X0, t1, t0, steps)
    h = fm.fm_flow_create([(kind, dev(A))], dtype, "tile=%dx%d;verbose=1" % (bm, bk))
    try:
        out = empty(N)
        fm.fm_fine_propagate(h, t1, t0, steps, [dev(X0)], [out])
        got = host(out)
    finally:
        fm.fm_destroy(h)
    _check_forced(capfd, bm, bk)
    e = rel(got, ref)
    say("  rel err %.3e" % e)
    assert e <= TOL[dtype]


@pytest.mark.parametrize("dtype,bm,bk", CASES)
def test_coarse_propagate_every_tile(dtype, bm, bk, capfd):
    from paper_1505_07959_amd import fm
    say("tile %dx%d dtype=%s n=%d coarse" % (bm, bk, dtype, N))
    A, X0 = _case(12)
    t0, t1, steps = 0.0, 0.2, 3
    ref = integrators.coarse(MatrixAlgebra(N), HOMOTOPY, A, X0, t1, t0, steps)
    h = fm.fm_flow_create([(HOMOTOPY, dev(A))], dtype, "tile=%dx%d;verbose=1" % (bm, bk))
    try:
        out = empty(N)
        fm.fm_coarse_propagate(h, t1, t0, steps, fm.FM_COARSE_EULER, [dev(X0)], [out])
        got = host(out)
    finally:
        fm.fm_destroy(h)
    _check_forced(capfd, bm, bk)
    e = rel(got, ref)
    say("  rel err %.3e" % e)
    assert e <= TOL[dtype]


@pytest.mark.parametrize("dtype,tile", [("f64", "256x64"), ("bf16", "128x16"), ("f16", "64"), ("f32", "256x32")])
def test_unknown_tile_is_rejected(dtype, tile):
    from paper_1505_07959_amd import fm
    say("tile option %s dtype=%s (not compiled) is rejected" % (tile, dtype))
    A, _ = _case(13)
    with pytest.raises(fm.FmError) as ei:
        fm.fm_flow_create([(HOMOTOPY, dev(A))], dtype, "tile=" + tile)
    assert ei.value.status == fm.FM_ERR_INVALID


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16", "bf16x3"])
def test_padding_leaves_products_bitwise_unchanged(dtype):
    """n = 300 padded to 320, 384 or 512 (option pad=64|128|256): every tile
    sums over k in the same 16- or 4-wide chunks in the same order, and the
    extra chunks are zero, so the fine propagation is bitwise identical."""
    from paper_1505_07959_amd import fm
    import numpy as np
    n = 300
    say("padding invariance dtype=%s n=%d" % (dtype, n))
    A, _, _ = inputs.spd(n, "uniform", 0.3, 2.0, 21)
    X0 = inputs.perturbed_identity(n, 121, eps=0.1)
    outs = []
    for pad in (64, 128, 256):
        h = fm.fm_flow_create([(HOMOTOPY, dev(A))], dtype, "pad=%d" % pad)
        try:
            out = empty(n)
            fm.fm_fine_propagate(h, 0.3, 0.1, 3, [dev(X0)], [out])
            outs.append(host(out))
        finally:
            fm.fm_destroy(h)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_unknown_padding_is_rejected():
    from paper_1505_07959_amd import fm
    A, _ = _case(13)
    with pytest.raises(fm.FmError) as ei:
        fm.fm_flow_create([(HOMOTOPY, dev(A))], "f64", "pad=96")
    assert ei.value.status == fm.FM_ERR_INVALID


@pytest.mark.parametrize("dtype", sorted(TILES))
def test_every_tile_gives_bitwise_identical_products(dtype):
    """All compiled tiles of a product type walk the same k-chunks in the
    same order, so their fine propagations agree bit for bit (the autotuner
    changes speed only)."""
    from paper_1505_07959_amd import fm
    import numpy as np
    say("tile bitwise invariance dtype=%s n=%d" % (dtype, N))
    A, X0 = _case(11)
    outs = []
    for bm, bk in TILES[dtype]:
        h = fm.fm_flow_create([(INV_LINEAR, dev(A))], dtype, "tile=%dx%d" % (bm, bk))
        try:
            out = empty(N)
            fm.fm_fine_propagate(h, 0.3, 0.1, 3, [dev(X0)], [out])
            outs.append(host(out))
        finally:
            fm.fm_destroy(h)
    for (bm, bk), o in zip(TILES[dtype][1:], outs[1:]):
        assert np.array_equal(outs[0], o), "tile %dx%d differs from %dx%d" % (bm, bk, *TILES[dtype][0])
