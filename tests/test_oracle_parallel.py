"""The row-parallel oracle runner (oracle/parallel.py) and the full-batch comparison
helpers (tests/fullsize.py) on the CPU: chunks come back in order, payloads reach their
chunk, and the chunked result equals the oracle on the whole batch."""
import numpy as np

import fullsize
from oracle import parallel, tabnet as ot
from paper_2510_19689_amd import synth


def _rows_and_payload(params, X, payload):
    return X.shape[0], payload, float(X[0, 0])


def _forward(params, X, payload):
    return ot.forward(params, X)


def test_map_rows_order_and_payload():
    p, X = synth.workload("hr35", rows=1000)
    got = list(parallel.map_rows(_rows_and_payload, p, X, chunk=300, workers=3, payload=lambda lo, hi: (lo, hi)))
    assert [g[0] for g in got] == [0, 300, 600, 900]
    assert [g[1][0] for g in got] == [300, 300, 300, 100]
    assert [g[1][1] for g in got] == [(0, 300), (300, 600), (600, 900), (900, 1000)]
    assert [g[1][2] for g in got] == [float(X[k, 0]) for k in (0, 300, 600, 900)]


def test_chunked_forward_equals_whole_batch():
    p, X = synth.workload("adult108", rows=700)
    ref = ot.forward(p, X)
    parts = [r for _, r in parallel.map_rows(_forward, p, X, chunk=256, workers=2)]
    for k in range(3):
        got = np.concatenate([q[k] for q in parts], axis=1 if k == 2 else 0)
        np.testing.assert_allclose(got, ref[k], rtol=1e-12, atol=1e-14)


def test_all_rows_reports_a_planted_error():
    """The per-row comparison finds one perturbed mask row among correct ones, and an
    argmax flip, and nothing else."""
    p, X = synth.workload("hr35", rows=600)
    lo, ag, ms = (np.asarray(a, dtype=np.float32) for a in ot.forward(p, X))
    ms2 = ms.copy()
    ms2[1, 417, 3] += 0.25
    lo2 = lo.copy()
    lo2[5] = lo2[5, ::-1]
    outs = {"a": (lo, ag, ms), "b": (lo2, ag, ms2)}
    fetch = lambda a, b: {k: (v[0][a:b], v[1][a:b], v[2][:, a:b]) for k, v in outs.items()}
    e = fullsize.all_rows(p, X, fetch, [("a", "a", None, None), ("b", "b", None, None)], chunk=128, workers=2,
                          say=None)
    sa, sb = fullsize.summary(e["a"]), fullsize.summary(e["b"])
    assert sa["step_l1"] < 1e-6 and sa["argmax"] == 1.0
    assert np.argmax(e["b"]["step_l1"]) == 417 and abs(sb["step_l1"] - 0.25) < 1e-6
    assert (e["b"]["step_l1"] > 1e-6).sum() == 1
    assert sb["argmax"] == 1.0 - 1.0 / 600 and not e["b"]["argmax"][5]
