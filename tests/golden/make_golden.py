"""Write oracle values too slow to recompute in a test run.

tests/golden/expected.json: whole-simplex checksums at full sizes, the
Axilrod-Teller + LJ energy and sampled gradient rows of the n = 8192 workload.
tests/golden/grad_n8192.npz (--full-grad): the oracle's full FP64 gradient
of that workload, Axilrod-Teller ("at", all C(8192, 3) triplets) and
Lennard-Jones ("lj") separately, each [8192, 3].

Calls only the oracle and the seeded input generators:
    python tests/golden/make_golden.py             # expected.json
    python tests/golden/make_golden.py --full-grad # grad_n8192.npz (minutes)
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "expected.json")
OUT_GRAD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_n8192.npz")

# sampled particles of the n = 8192 gradient check: tile edges of 32 and 64,
# both ends, plus seeded random picks
GRAD_ROWS = sorted({0, 1, 31, 32, 63, 64, 4095, 4096, 8190, 8191,
                    *np.random.default_rng(99).integers(0, 8192, 10).tolist()})


def sha(x: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest()


def main():
    res = {"inputs": {}, "checksums": {}, "at_lj_n8192": {}}
    t0 = time.time()
    for name in synth.WORKLOADS:
        x = synth.workload_input(name)
        res["inputs"][name] = {"shape": list(x.shape), "sha256": sha(x)}
    print("inputs hashed", time.time() - t0, flush=True)
    # whole-simplex checksums (wrapping uint64, stored as decimal strings)
    vols = {
        "pairs_le_65536": oracle.simplex_volume(2, 65536, False),
        "pairs_le_32768": oracle.simplex_volume(2, 32768, False),
        "pairs_lt_8192": oracle.simplex_volume(2, 8192, True),
        "triplets_lt_2048": oracle.simplex_volume(3, 2048, True),
        "triplets_lt_8192": oracle.simplex_volume(3, 8192, True),
        "triplets_le_8192": oracle.simplex_volume(3, 8192, False),
    }
    for k, v in vols.items():
        res["checksums"][k] = {"volume": v, "checksum": str(oracle.checksum_range(v))}
        print(k, v, time.time() - t0, flush=True)
    X = synth.workload_input("at_lj_n8192")
    g = res["at_lj_n8192"]
    g["lj_energy"] = oracle.lj_energy(X, 1.0, 1.0, 3.0)
    g["grad_rows"] = GRAD_ROWS
    g["at_grad_rows"] = oracle.at_grad_rows(X, GRAD_ROWS, 1.0).tolist()
    g["lj_grad_rows"] = oracle.lj_grad(X, 1.0, 1.0, 3.0)[GRAD_ROWS].tolist()
    print("grad rows", time.time() - t0, flush=True)
    g["at_energy"] = oracle.at_energy(X, 1.0)
    g["oracle_threads"] = oracle.threads()
    print("at energy", g["at_energy"], time.time() - t0, flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


def full_grad():
    X = synth.workload_input("at_lj_n8192")
    t0 = time.time()
    at = oracle.at_grad(X, 1.0)
    print("at grad", time.time() - t0, flush=True)
    lj = oracle.lj_grad(X, 1.0, 1.0, 3.0)
    np.savez(OUT_GRAD, at=at, lj=lj, input_sha256=np.array(sha(X)))
    print("wrote", OUT_GRAD, "threads", oracle.threads())


if __name__ == "__main__":
    if "--full-grad" in sys.argv[1:]:
        full_grad()
    else:
        main()
