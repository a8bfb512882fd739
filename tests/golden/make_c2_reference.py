"""Write tests/golden/c2_reference.json: the FP64 oracle's results on the 512^3 headline
workload (planted rank-10 tensor, factors U[0,1) zeroed w.p. 0.5, U[0,1e-3) noise, seed 2,
stored FP32; nnTucker multirank (20,20,20) for 500 multiplicative-update sweeps from the
seeded U[0,1) initial values; nnCP rank 10 of the core for 300 sweeps; lift).

Calls only the oracle and the seeded input generator.  Takes several CPU-minutes.
    python tests/golden/make_c2_reference.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

SEED, N, R, RANK, SWEEPS, CP_SWEEPS = 2, 512, 20, 10, 500, 300


def main():
    t0 = time.time()
    X32, _ = synth.planted_tensor(SEED, (N, N, N), 10, zero_prob=0.5, noise=1e-3, dtype="f32")
    X = X32.astype(np.float64)
    del X32
    G0 = synth.init_core(SEED, (R, R, R)).astype(np.float64)
    A0 = [a.astype(np.float64) for a in synth.init_factors(SEED, (N, N, N), (R, R, R))]
    B0 = [b.astype(np.float64) for b in synth.init_cp_factors(SEED, (R, R, R), RANK)]
    G1, A1, _, _ = oracle.nntucker(X, G0, A0, 1)
    one = {"tucker_rel": oracle.tucker_rel_residual(X, G1, A1),
           "core_fro": float(np.linalg.norm(G1)),
           "factor_fro": [float(np.linalg.norm(a)) for a in A1]}
    G, A, clips, _ = oracle.nntucker(X, G0, A0, SWEEPS)
    tucker_rel = oracle.tucker_rel_residual(X, G, A)
    B, _, _ = oracle.nncp(G, B0, CP_SWEEPS)
    C = oracle.lift(A, B)
    cp_rel = oracle.cp_rel_residual(X, C)
    out = {"about": "FP64 oracle on the 512^3 headline workload (see the docstring of make_c2_reference.py)",
           "seed": SEED, "dims": [N, N, N], "multirank": [R, R, R], "sweeps": SWEEPS,
           "cp_rank": RANK, "cp_sweeps": CP_SWEEPS, "clips": clips,
           "after_one_sweep": one, "tucker_rel": tucker_rel, "cp_rel": cp_rel,
           "threads": oracle.get_threads(), "seconds": time.time() - t0}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_reference.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
