"""Tile sweep of each compiled shape family.

The tiling of a shape is fixed at build time: the register-resident kernel carries R
16-row blocks per wavefront and W wavefronts per workgroup (the weight chunks are sized
from both); the split-feature kernel shares the features of 16 rows over W wavefronts and
holds RG such groups per workgroup.  R, W of the register-resident kernel and RG never
change a row's arithmetic, so those candidates must give the product library's outputs bit
for bit; W of the split-feature kernel regroups the per-wave partial sums of a row (the
sparsemax and the decision sums), so its candidates agree to FP32 rounding.

    python -m paper_2510_19689_amd.tile_sweep build [family ...]  # one library per candidate (CPU)
    python -m paper_2510_19689_amd.tile_sweep run [family ...]   # time them on the GPU

`run` times each candidate in a process of its own (the library is chosen by TABNET_LIB),
interleaving the product tiling before and after the family's candidates, and prints one
markdown table per family with the time per launch and whether the outputs match.
"""
from __future__ import annotations

import hashlib
import json
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "_build", "tile_sweep")

# family -> workload, rows timed, the compiled shape (prec, DT, NT, KA0), the product
# tiling and the candidates: (R, W) for the register-resident kernel, (W, RG) for the
# split-feature one.
FAMILIES = {
    "hr35": dict(workload="hr35", rows=65536, shape=(1, 3, 1, 0), wide=False, product=(1, 4),
                 candidates=[(1, 1), (1, 2), (1, 4), (1, 8), (1, 16), (2, 4)]),
    "adult108": dict(workload="adult108", rows=65536, shape=(1, 7, 4, 2), wide=False, product=(1, 8),
                     candidates=[(1, 2), (1, 4), (1, 8), (1, 12), (1, 16), (2, 4), (2, 8)]),
    "wide200": dict(workload="wide200", rows=262144, shape=(1, 13, 8, 4), wide=False, product=(1, 8),
                    candidates=[(1, 1), (1, 2), (1, 4), (1, 8), (2, 2)]),
    "wide512": dict(workload="wide512", rows=65536, shape=(1, 32, 8, 4), wide=True, product=(4, 2),
                    candidates=[(2, 1), (2, 2), (2, 3), (4, 1), (4, 2), (4, 3)]),
}
# the 200-feature shape on the split-feature kernel
FAMILIES["wide200_split"] = dict(workload="wide200", rows=262144, shape=(1, 13, 8, 4), wide=True, product=None,
                                 candidates=[(2, 1), (2, 2), (2, 4), (4, 1), (4, 2)])
# the 200-feature shape in the other precisions: one or two waves per SIMD
PREC_CODES = {"fp32": 0, "fp8": 2, "int8": 3, "mxfp8": 4, "mxfp4": 5, "mxfp6": 6, "mxfp8_e5m2": 7,
              "mxfp6_e3m2": 8, "fp8w": 9}
for _p, _c in PREC_CODES.items():
    FAMILIES[f"wide200_{_p}"] = dict(workload="wide200", rows=262144, shape=(_c, 13, 8, 4), wide=False,
                                     product=(1, 8) if _c in (0, 2, 5, 9) else (1, 4),
                                     candidates=[(1, 4), (1, 8)], prec=_p)


def _entry(fam: dict, t) -> str:
    p, dt, nt, ka0 = fam["shape"]
    if fam["wide"]:
        return f"TABNET_WIDE_SHAPE({p},{dt},{nt},{ka0},{t[0]},{t[1]})"
    return f"TABNET_SHAPE({p},{dt},{nt},{ka0},{t[0]},{t[1]})"


def _lib(name: str, t) -> str:
    return os.path.join(OUT, f"{name}_{t[0]}x{t[1]}.so")


def build_all(families=None, jobs: int = 4) -> None:
    from paper_2510_19689_amd import build as B
    os.makedirs(OUT, exist_ok=True)
    work = [(name, t) for name in (families or FAMILIES) for t in FAMILIES[name]["candidates"]]

    def one(nt):
        name, t = nt
        B.build_variant([f"TABNET_TILE_SWEEP={_entry(FAMILIES[name], t)}"], _lib(name, t))
        return name, t

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for name, t in ex.map(one, work):
            print(f"built {name} {t}", flush=True)


def _child(lib: str, workload: str, rows: int, sample: str, prec: str) -> None:
    """Time one library on one workload (step masks on); prints a JSON line and saves the
    outputs of the first 1,024 rows to `sample` (.npz)."""
    os.environ["TABNET_LIB"] = lib
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch
    from paper_2510_19689_amd import synth, tabnet as tb
    params, X = synth.workload(workload, rows=rows)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.tnw")
        synth.write_weights(params, path)
        with tb.Model(path, prec) as m:
            Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
            lo, ag, ms = m.outputs(rows, True)
            m.forward_into(Xd, lo, ag, ms)
            torch.cuda.synchronize()
            digest = hashlib.sha256()
            for t in (lo, ag, ms):
                digest.update(t.cpu().numpy().tobytes())
            k = min(rows, 1024)
            np.savez(sample, lo=lo[:k].cpu().numpy(), ag=ag[:k].cpu().numpy(), ms=ms[:, :k].cpu().numpy())
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            m.forward_into(Xd, lo, ag, ms)
            e1.record()
            torch.cuda.synchronize()
            n = max(5, int(0.2e3 / max(e0.elapsed_time(e1), 1e-3)))   # about 0.2 s per repetition
            for _ in range(2 * n):
                m.forward_into(Xd, lo, ag, ms)
            torch.cuda.synchronize()
            reps = []
            for _ in range(3):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(n):
                    m.forward_into(Xd, lo, ag, ms)
                e1.record()
                torch.cuda.synchronize()
                reps.append(e0.elapsed_time(e1) / n * 1e3)
    print(json.dumps({"us": min(reps), "reps": reps, "sha": digest.hexdigest()[:16]}), flush=True)


def _time(lib: str, workload: str, rows: int, sample: str, prec: str) -> dict:
    r = subprocess.run([sys.executable, "-m", "paper_2510_19689_amd.tile_sweep", "child", lib, workload, str(rows),
                        sample, prec], capture_output=True, text=True, cwd=ROOT, timeout=300)
    if r.returncode != 0:
        return {"error": (r.stderr.strip().splitlines() or ["exit %d" % r.returncode])[-1]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def _maxdiff(a: str, b: str) -> float:
    import numpy as np
    x, y = np.load(a), np.load(b)
    return max(float(np.abs(x[k].astype(np.float64) - y[k]).max()) for k in ("lo", "ag", "ms"))


def run_all(families=None) -> None:
    product = os.path.join(HERE, "libtabnet.so")
    tmp = tempfile.mkdtemp(prefix="tile_sweep_")
    for name in families or FAMILIES:
        fam = FAMILIES[name]
        wl, rows, prec = fam["workload"], fam["rows"], fam.get("prec", "bf16")
        print(f"[sweep] {name}: {wl}, {rows} rows, {prec}, step masks on", file=sys.stderr, flush=True)
        ref_npz = os.path.join(tmp, f"{name}_product.npz")
        ref0 = _time(product, wl, rows, ref_npz, prec)
        res = {}
        for t in fam["candidates"]:
            npz = os.path.join(tmp, f"{name}_{t[0]}x{t[1]}.npz")
            res[t] = _time(_lib(name, t), wl, rows, npz, prec)
            if "error" not in res[t] and "error" not in ref0:
                res[t]["maxdiff"] = _maxdiff(npz, ref_npz)
            print(f"[sweep] {name} {t}: {res[t]}", file=sys.stderr, flush=True)
        ref1 = _time(product, wl, rows, os.path.join(tmp, f"{name}_product2.npz"), prec)
        a, b = ("R", "W") if not fam["wide"] else ("W", "RG")
        prod = f"{a}={fam['product'][0]}, {b}={fam['product'][1]}" if fam["product"] else "another kernel"
        print(f"\n{name} ({wl}, {rows:,} rows, {prec}, step masks on); product tiling {prod}: "
              f"{ref0.get('us', float('nan')):.1f} us before the candidates, "
              f"{ref1.get('us', float('nan')):.1f} us after\n")
        print(f"| {a} | {b} | us per launch | all outputs bit-equal to the product's | max diff, first 1,024 rows |")
        print("|---|---|---|---|---|")
        for t, r in res.items():
            if "error" in r:
                print(f"| {t[0]} | {t[1]} | failed: {r['error'][:80]} | | |")
                continue
            same = "yes" if r["sha"] == ref0.get("sha") else "no"
            mark = " (product)" if fam["product"] and t == tuple(fam["product"]) else ""
            print(f"| {t[0]} | {t[1]}{mark} | {r['us']:.1f} | {same} | {r.get('maxdiff', float('nan')):.3g} |")
        sys.stdout.flush()


if __name__ == "__main__":
    cmd = sys.argv[1] if len(sys.argv) > 1 else "run"
    if cmd == "build":
        build_all(sys.argv[2:] or None)
    elif cmd == "child":
        _child(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], sys.argv[6])
    else:
        run_all(sys.argv[2:] or None)
