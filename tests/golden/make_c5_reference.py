"""Write tests/golden/c5_reference.json and c5_core.npy: the FP64 oracle's results on the
64^5 workload (planted rank-6 tensor, factors U[0,1), U[0,1e-3) noise, seed 5, stored FP32;
nnTucker multirank (8,8,8,8,8) for 300 multiplicative-update sweeps from the seeded U[0,1)
initial values), and 64 random-restart nnCP fits of the fitted core: restart j has rank
2 + (j mod 15) and its own seeded U[0,1) initial factors, 300 sweeps each.

c5_core.npy holds the oracle's fitted core rounded to float32.  The 64 restarts run on that
rounded core, so that a GPU batched nnCP can start from the identical input; the JSON holds
each restart's relative residual ||core - cp(B)||_F / ||core||_F and the lifted model's
relative error against X for restart 0.

Calls only the oracle and the seeded input generator.  About 1-2 CPU-hours on 8 cores and
about 22 GB of memory.
    python tests/golden/make_c5_reference.py
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

SEED, N, D, PLANTED, R, SWEEPS, CP_SWEEPS, RESTARTS = 5, 64, 5, 6, 8, 300, 300, 64
HERE = os.path.dirname(os.path.abspath(__file__))


def restart_rank(j):
    return 2 + (j % 15)


def main():
    t0 = time.time()
    dims, ranks = (N,) * D, (R,) * D
    X32, _ = synth.planted_tensor(SEED, dims, PLANTED, noise=1e-3, dtype="f32")
    X = X32.astype(np.float64)
    del X32
    G0 = synth.init_core(SEED, ranks).astype(np.float64)
    A0 = [a.astype(np.float64) for a in synth.init_factors(SEED, dims, ranks)]
    G, A, clips, _ = oracle.nntucker(X, G0, A0, SWEEPS)
    t_tucker = time.time() - t0
    tucker_rel = oracle.tucker_rel_residual(X, G, A)
    core32 = G.astype(np.float32)
    np.save(os.path.join(HERE, "c5_core.npy"), core32)
    core = core32.astype(np.float64)
    rels, cp_clips = [], 0
    B_first = None
    for j in range(RESTARTS):
        B0 = synth.init_cp_factors(SEED, ranks, restart_rank(j), restart=j)
        B, c, _ = oracle.nncp(core, B0, CP_SWEEPS)
        cp_clips += c
        rels.append(oracle.cp_rel_residual(core, B))
        if j == 0:
            B_first = B
    lifted_rel0 = oracle.cp_rel_residual(X, oracle.lift(A, B_first))
    out = {"about": "FP64 oracle on the 64^5 workload (see the docstring of make_c5_reference.py)",
           "seed": SEED, "dims": list(dims), "planted_rank": PLANTED, "multirank": list(ranks),
           "sweeps": SWEEPS, "clips": clips, "tucker_rel": tucker_rel,
           "core_npy": "c5_core.npy", "cp_sweeps": CP_SWEEPS,
           "restart_ranks": [restart_rank(j) for j in range(RESTARTS)],
           "restart_core_rel": rels, "restart_clips": cp_clips,
           "restart0_lifted_rel": lifted_rel0,
           "threads": oracle.get_threads(), "tucker_seconds": t_tucker,
           "seconds": time.time() - t0}
    with open(os.path.join(HERE, "c5_reference.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
