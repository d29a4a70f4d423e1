"""peps_evaluate_noalloc (workspace in the library's fixed device scratch array) against
peps_evaluate (allocated workspace), through the C ABI, on two calls in a row, the
second with a smaller batch, so the second call runs on what the first left in the
array.  Per-sample outputs (log-amplitude, sign, local energy, flags, per-sample
log-derivatives) must be equal bit for bit: the kernels are the same and every sample
is computed independently of the chunk it falls in.  The Eq. (5) gradient sums over the
batch in per-chunk partitions, and the two entry points may cut the batch into
different chunks, so those sums are compared at 1e-12 of their norm."""
import sys

import numpy as np
import pytest

from paper_1806_03761_amd.workloads import Lattice, make_random, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _peps():
    from paper_1806_03761_amd import peps
    return peps


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _run(peps, A, S, lat, prec, grad_mode, noalloc, weights=None):
    r = peps.evaluate(A, S, lat, prec, grad_mode=grad_mode, weights=weights, noalloc=noalloc)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in r]


def _compare(a, b, grad_mode):
    la0, sg0, e0, g0, f0 = a
    la1, sg1, e1, g1, f1 = b
    for name, x, y in (("log-amp", la0, la1), ("sign", sg0, sg1), ("E_loc", e0, e1), ("flags", f0, f1)):
        assert np.array_equal(x, y, equal_nan=True), name
    if grad_mode == 1:
        assert np.array_equal(g0, g1)
    elif grad_mode in (2, 3):
        scale = max(np.linalg.norm(g0), 1e-300)
        assert np.linalg.norm(g1 - g0) <= 1e-12 * scale, float(np.linalg.norm(g1 - g0) / scale)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_matches_evaluate_4x4(prec):
    peps = _peps()
    lat, A, S, _ = make_workload("4x4_D2_Dc4")
    Ad = torch.from_numpy(A).cuda()
    for n, gm in ((256, 3), (37, 1)):
        Sd = torch.from_numpy(np.ascontiguousarray(S[:n])).cuda()
        _say("noalloc 4x4 D2 Dc4", prec, "batch", n, "grad_mode", gm)
        ref = _run(peps, Ad, Sd, lat, prec, gm, False)
        got = _run(peps, Ad, Sd, lat, prec, gm, True)
        _compare(ref, got, gm)


def test_noalloc_with_variational_compression():
    """With the context's truncation set to variational compression the allocation-free
    entry point keeps the compression's environments and temporaries in the fixed array
    too: per-sample results equal peps_evaluate's bit for bit on two calls in a row."""
    peps = _peps()
    lat = Lattice(6, 6, 3, 5)
    A, S = make_random(lat, 64, 46)
    Ad = torch.from_numpy(A).cuda()
    peps.set_truncation(1)
    try:
        for n in (64, 21):
            Sd = torch.from_numpy(np.ascontiguousarray(S[:n])).cuda()
            _say("noalloc variational 6x6 D3 Dc5, batch", n)
            ref = _run(peps, Ad, Sd, lat, "f64", 1, False)
            got = _run(peps, Ad, Sd, lat, "f64", 1, True)
            _compare(ref, got, 1)
    finally:
        peps.set_truncation(0)


def test_noalloc_chunks_8x8_and_ignores_workspace_limit():
    """8x8, D = 4, Dc = 16 needs about 3.2 MiB for one sample and 2.2 MiB for each more,
    so 40 samples exceed the 64 MiB array and run in two chunks; then 9 samples.  With
    the context's workspace limit set to 1 MiB the allocating entry point refuses the
    batch while the allocation-free one, which never uses that workspace, still runs."""
    peps = _peps()
    lat, A, S, _ = make_workload("8x8_D4_Dc16", 40)
    A2, S2 = make_random(lat, 91, 92, "half")
    S = np.concatenate([S[:31], S2[:9]])
    Ad = torch.from_numpy(A).cuda()
    assert peps.noalloc_scratch_bytes() == 64 << 20
    assert peps.workspace_bytes(lat, 40) > peps.noalloc_scratch_bytes()
    for n, gm, w in ((40, 3, None), (9, 2, np.linspace(-1.0, 2.0, 9))):
        Sd = torch.from_numpy(np.ascontiguousarray(S[:n])).cuda()
        wd = torch.from_numpy(w).cuda() if w is not None else None
        _say("noalloc 8x8 D4 Dc16 f64 batch", n, "grad_mode", gm)
        ref = _run(peps, Ad, Sd, lat, "f64", gm, False, wd)
        try:
            peps.set_workspace_limit(1 << 20)
            with pytest.raises(peps.PepsError):
                peps.evaluate(Ad, Sd, lat, "f64", grad_mode=gm, weights=wd)
            got = _run(peps, Ad, Sd, lat, "f64", gm, True, wd)
        finally:
            peps.set_workspace_limit(0)
        _compare(ref, got, gm)


def test_noalloc_rejects_a_sample_beyond_the_array():
    """16x16, D = 6, Dc = 36 needs about 91 MiB for one sample: refused on the host with
    a message naming the fixed scratch, before any kernel runs."""
    peps = _peps()
    lat = Lattice(16, 16, 6, 36)
    A, S = make_random(lat, 5, 6, "half")
    Ad, Sd = torch.from_numpy(A).cuda(), torch.from_numpy(np.ascontiguousarray(S[:2])).cuda()
    _say("noalloc 16x16 D6 Dc36 refusal")
    with pytest.raises(peps.PepsError, match="fixed scratch"):
        peps.evaluate(Ad, Sd, lat, "f64", grad_mode=3, noalloc=True)
