"""Write tests/golden/c3_reference.json and c3_core.npy: the FP64 oracle's results on the
128^4 workload stored as bfloat16 (planted rank-8 tensor, factors U[0,1), U[0,1e-3) noise,
seed 3, every entry rounded once to bf16 (RNE); nnTucker multirank (16,16,16,16) for 500
multiplicative-update sweeps from the seeded U[0,1) initial values; nnCP rank 8 of the core
for 300 sweeps; lift).

The oracle reads the bf16 values widened exactly to float64, which is also what the GPU's FP32
form and its FP32 refinement sweeps read.  c3_core.npy holds the oracle's fitted core rounded
to float32, and the JSON the oracle's nnCP of that rounded core, so that a GPU nnCP can start
from the identical input.

Calls only the oracle and the seeded input generator.  About 25-45 CPU-minutes on 8 cores.
    python tests/golden/make_c3_reference.py
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

SEED, N, D, PLANTED, R, RANK, SWEEPS, CP_SWEEPS = 3, 128, 4, 8, 16, 8, 500, 300
HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    t0 = time.time()
    dims, ranks = (N,) * D, (R,) * D
    bits, _ = synth.planted_tensor(SEED, dims, PLANTED, noise=1e-3, dtype="bf16")
    X = synth.bf16_bits_to_f64(bits)
    del bits
    G0 = synth.init_core(SEED, ranks).astype(np.float64)
    A0 = [a.astype(np.float64) for a in synth.init_factors(SEED, dims, ranks)]
    B0 = [b.astype(np.float64) for b in synth.init_cp_factors(SEED, ranks, RANK)]
    G, A, clips, _ = oracle.nntucker(X, G0, A0, SWEEPS)
    t_tucker = time.time() - t0
    tucker_rel = oracle.tucker_rel_residual(X, G, A)
    B, cp_clips, _ = oracle.nncp(G, B0, CP_SWEEPS)
    C = oracle.lift(A, B)
    cp_rel = oracle.cp_rel_residual(X, C)
    core32 = G.astype(np.float32)
    np.save(os.path.join(HERE, "c3_core.npy"), core32)
    Bc, cpc_clips, _ = oracle.nncp(core32.astype(np.float64), B0, CP_SWEEPS)
    core_cp_rel = oracle.cp_rel_residual(core32, Bc)
    out = {"about": "FP64 oracle on the 128^4 bf16 workload (see the docstring of make_c3_reference.py)",
           "seed": SEED, "dims": list(dims), "planted_rank": PLANTED, "multirank": list(ranks),
           "sweeps": SWEEPS, "cp_rank": RANK, "cp_sweeps": CP_SWEEPS, "clips": clips + cp_clips,
           "tucker_rel": tucker_rel, "cp_rel": cp_rel,
           "core_npy": "c3_core.npy", "core_cp_rel": core_cp_rel, "core_cp_clips": cpc_clips,
           "threads": oracle.get_threads(), "tucker_seconds": t_tucker,
           "seconds": time.time() - t0}
    with open(os.path.join(HERE, "c3_reference.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
