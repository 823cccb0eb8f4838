"""redsea_trsm_noalloc (scratch in a fixed device array, no allocation)
against redsea_trsm with the same schedule: bitwise equal results on two
calls in a row, the second smaller, so the array's leftover contents from
the first call must not leak into the second; the size limit is enforced
before any device work; a captured graph of the call replays correctly."""
import sys

import numpy as np
import pytest

import oracle
import paper_2305_19917_amd as rs
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _both(L, B, **kw):
    dL = rs.fortran_tensor(L)
    d1, d2 = rs.fortran_tensor(B), rs.fortran_tensor(B)
    rs.trsm(dL, d1, precision="native", **kw)
    rs.trsm_noalloc(dL, d2, **kw)
    torch.cuda.synchronize()
    return d1.cpu().numpy(), d2.cpu().numpy()


@pytest.mark.parametrize("variant,nb", [("recursive", 256), ("iterative", 128), ("blocked", 64)])
def test_noalloc_matches_trsm_big_then_small(variant, nb):
    for k, nrhs, key in [(3000, 300, (24, 0)), (700, 90, (24, 1))]:
        _say("noalloc", variant, nb, k, nrhs)
        L = synth.dominant_lower(k, key + (0,))
        B = synth.rhs_normal(k, nrhs, key + (1,))
        X1, X2 = _both(L, B, variant=variant, nb=nb)
        assert np.array_equal(X1, X2), (variant, nb, k)
        assert oracle.backward_error(0, 0, 0, 0, 1.0, L, B, X2) <= 1e-14 * k


def test_noalloc_flags_alpha_fp32():
    k, nrhs = 517, 33
    L = synth.dominant_lower(k, (25, 0, 0))
    for side, uplo, trans, diag in [(0, 1, 1, 0), (1, 0, 0, 1), (1, 1, 1, 0)]:
        A = np.asfortranarray(L if uplo == 0 else L.T)
        B = synth.rhs_normal(*((k, nrhs) if side == 0 else (nrhs, k)), key=(25, side, 1))
        X1, X2 = _both(A, B, side=side, uplo=uplo, trans=trans, diag=diag, alpha=-1.5,
                       variant="recursive", nb=128)
        assert np.array_equal(X1, X2)
    B = synth.rhs_normal(k, nrhs, (25, 9, 1))
    X1, X2 = _both(L.astype(np.float32), B.astype(np.float32), variant="recursive", nb=256)
    assert np.array_equal(X1, X2)


def test_noalloc_rejects_oversize_and_refinement():
    # FP64 order 12288 at nb 256 needs 48 packed blocks of 770 KB > 32 MiB:
    # refused on the host before anything touches the (never allocated) data
    L = rs.lib()
    opts = rs.Opts(1, 256, 1)
    import ctypes
    rc = L.redsea_trsm_noalloc(0, 0, 0, 0, 0, 12288, 4, 1.0, 8, 12288, 8, 12288,
                               ctypes.byref(opts), None)
    assert rc == 6 and "scratch" in rs.status_string(rc)
    opts = rs.Opts(1, 256, 2)
    assert L.redsea_trsm_noalloc(0, 0, 0, 0, 0, 100, 4, 1.0, 8, 100, 8, 100,
                                 ctypes.byref(opts), None) == 5
    # the largest FP64 order it takes at nb 256 (43 blocks) still solves
    # (300 right-hand sides: the split schedule with its packed blocks)
    k, nrhs = 43 * 256, 300
    Lh = synth.dominant_lower(k, (26, 0, 0))
    B = synth.rhs_normal(k, nrhs, (26, 0, 1))
    X1, X2 = _both(Lh, B, variant="recursive", nb=256)
    assert np.array_equal(X1, X2)


def test_noalloc_thin_big_then_small_and_captured():
    # few right-hand sides: the one-launch solve, its flags in the array
    for k, nrhs, key in [(3000, 8, (28, 0)), (700, 3, (28, 1)), (5000, 32, (28, 2))]:
        _say("noalloc thin", k, nrhs)
        L = synth.dominant_lower(k, key + (0,))
        B = synth.rhs_normal(k, nrhs, key + (1,))
        rs.trace_begin()
        X1, X2 = _both(L, B, variant="recursive", nb=256)
        assert rs.trace_end()["thin"][0] == 2
        assert np.array_equal(X1, X2), k
        assert oracle.backward_error(0, 0, 0, 0, 1.0, L, B, X2) <= 1e-14 * k
    k, nrhs = 2500, 6
    L = synth.dominant_lower(k, (28, 3, 0))
    B = synth.rhs_normal(k, nrhs, (28, 3, 1))
    dL, dB0 = rs.fortran_tensor(L), rs.fortran_tensor(B)
    dB = dB0.clone()
    ref = dB0.clone()
    rs.trsm(dL, ref, variant="recursive", nb=256)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    rs.trsm_noalloc(dL, dB[:, :0])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    _say("noalloc thin capture")
    with torch.cuda.graph(g, stream=s):
        rs.trsm_noalloc(dL, dB, variant="recursive", nb=256, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        X1, X2 = _both(synth.dominant_lower(900, (28, 4, 0)), synth.rhs_normal(900, 5, (28, 4, 1)),
                       variant="recursive", nb=256)
        assert np.array_equal(X1, X2)
        dB.copy_(dB0)
        torch.cuda.synchronize()
        _say("noalloc thin replay", rep)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(dB.cpu().numpy(), ref), rep


def test_noalloc_graph_capture_and_replay():
    k, nrhs = 2000, 200
    L = synth.dominant_lower(k, (27, 0, 0))
    B = synth.rhs_normal(k, nrhs, (27, 0, 1))
    dL, dB0 = rs.fortran_tensor(L), rs.fortran_tensor(B)
    dB = dB0.clone()
    ref = dB0.clone()
    rs.trsm(dL, ref, variant="recursive", nb=256)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    # an empty call looks up the scratch array's address outside the capture
    rs.trsm_noalloc(dL, dB[:, :0])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rs.trsm_noalloc(dL, dB, variant="recursive", nb=256, stream=s)
    torch.cuda.synchronize()
    other = synth.rhs_normal(1200, 50, (27, 1, 1))
    for rep in range(3):
        # eager work in between reuses the scratch array with other contents
        X1, X2 = _both(synth.dominant_lower(1200, (27, 1, 0)), other, variant="blocked", nb=64)
        assert np.array_equal(X1, X2)
        dB.copy_(dB0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(dB.cpu().numpy(), ref), rep
