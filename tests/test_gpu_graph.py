"""Caller-side graph capture of the forward entry points.

A caller may capture tabnet_forward (or tabnet_forward_raw) and tabnet_mask_stats into one
HIP graph (here through torch.cuda.graph) and replay it: none of them allocates,
synchronises or writes memory with a memset node.  A graph captured once and replayed
several times, with input changes, poisoned outputs and unrelated eager launches between
the replays, must give on every replay exactly (bit for bit) the eager result for the
input it holds at that moment."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2510_19689_amd import synth, tabnet as tb  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    if not os.path.exists(tb.LIB_PATH):
        pytest.fail("libtabnet.so not built")


def _poison(*ts):
    for t in ts:
        t.fill_(float("nan"))


def _same(got, ref):
    for u, v in zip(got, ref):
        torch.testing.assert_close(u, v, rtol=0, atol=0, equal_nan=False)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "int8", "mxfp4"])
def test_forward_and_stats_graph_replays_equal_eager(tmp_path, prec):
    params, X1 = synth.workload("adult108", rows=2500)
    X2 = synth.make_inputs("adult", 2500, seed=77)
    X3 = synth.make_inputs("adult", 700, seed=78)
    path = str(tmp_path / "m.tnw")
    synth.write_weights(params, path)
    _say(f"case graph replay forward + mask stats {prec}")
    with tb.Model(path, prec) as m:
        refs = []
        for X in (X1, X2):
            out = m.forward(torch.from_numpy(X).cuda())
            refs.append(out + tb.mask_stats(out[1]))
        torch.cuda.synchronize()
        Xs = torch.from_numpy(X1).cuda()
        lo, ag, ms = m.outputs(2500, True)
        mean = torch.empty(108, dtype=torch.float64, device="cuda")
        var = torch.empty_like(mean)
        ws = torch.empty(max(tb.mask_stats_workspace_bytes(2500, 108), 1), dtype=torch.uint8, device="cuda")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            m.forward_into(Xs, lo, ag, ms)
            tb.mask_stats_into(ag, mean, var, ws)
        for k, (src, ref) in enumerate(((X1, refs[0]), (X2, refs[1]), (X1, refs[0]), (X2, refs[1]))):
            Xs.copy_(torch.from_numpy(src))
            _poison(lo, ag, ms, mean, var)
            other = m.forward(torch.from_numpy(X3).cuda())        # an unrelated eager launch
            g.replay()
            torch.cuda.synchronize()
            _same((lo, ag, ms, mean, var), ref)
            assert bool(torch.isfinite(other[0]).all())
            _say(f"replay {k} equals the eager result")


def test_raw_forward_graph_replays_equal_eager(tmp_path):
    """The same for the raw-row entry (embedding gathered in the kernel), BF16."""
    params, _ = synth.workload("adult108", rows=1)
    path = str(tmp_path / "m.tnw")
    synth.write_weights(params, path)
    X1, cards, dims, tables = synth.make_raw_inputs("adult", 1800, synth.DATA_SEED["adult108"])
    X2, _, _, _ = synth.make_raw_inputs("adult", 1800, 91)
    C = X1.shape[1]
    _say("case graph replay raw forward bf16")
    with tb.Model(path, "bf16") as m:
        m.set_embeddings(cards, dims, tables)
        refs = [m.forward_raw(torch.from_numpy(X).cuda()) for X in (X1, X2)]
        torch.cuda.synchronize()
        Xs = torch.from_numpy(X1).cuda()
        lo = torch.empty((1800, 2), dtype=torch.float32, device="cuda")
        ag = torch.empty((1800, C), dtype=torch.float32, device="cuda")
        ms = torch.empty((5, 1800, C), dtype=torch.float32, device="cuda")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            m.forward_raw_into(Xs, lo, ag, ms)
        for k, (src, ref) in enumerate(((X1, refs[0]), (X2, refs[1]), (X1, refs[0]))):
            Xs.copy_(torch.from_numpy(src))
            _poison(lo, ag, ms)
            g.replay()
            torch.cuda.synchronize()
            _same((lo, ag, ms), ref)
            _say(f"raw replay {k} equals the eager result")
