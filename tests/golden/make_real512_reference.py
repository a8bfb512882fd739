"""Write tests/golden/real512_reference.json, real512_factors.npz and real512_core.npy: the
FP64 oracle's real-valued CANDELINC (Section 2.2) on a 512^3 real tensor: a planted rank-20
CP with factor entries U[-1,1) plus U[-1e-3,1e-3) noise (synth.signed_planted, seed 7),
rounded once to float32; Tucker multirank (20,20,20) by 25 sweeps of alternating least squares
with orthonormalized factors from the seeded U[0,1) initial values; CP rank 20 of the core by
300 sweeps of alternating least squares from initial factors 2u - 1 (u the seeded nnCP
initial draws); lift.

real512_factors.npz holds the oracle's Tucker factors (float32) so that the GPU's factor
subspaces can be compared through their projectors; real512_core.npy the oracle's core
rounded to float32, from which the JSON's CP fit starts, so that a GPU CP fit can start from
the identical input.

Calls only the oracle and the seeded input generator.  About 5-10 CPU-minutes on 8 cores.
    python tests/golden/make_real512_reference.py
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

SEED, N, PLANTED, R, RANK, SWEEPS, CP_SWEEPS, NOISE = 7, 512, 20, 20, 20, 25, 300, 1e-3
HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    t0 = time.time()
    dims, ranks = (N,) * 3, (R,) * 3
    X, P = synth.signed_planted(SEED, dims, PLANTED, noise=NOISE)
    X = X.astype(np.float32).astype(np.float64)
    t_gen = time.time() - t0
    G0 = synth.init_core(SEED, ranks).astype(np.float64)
    A0 = [a.astype(np.float64) for a in synth.init_factors(SEED, dims, ranks)]
    B0 = [2.0 * b.astype(np.float64) - 1.0 for b in synth.init_cp_factors(SEED, ranks, RANK)]
    G, A, hist = oracle.tucker_ls(X, G0, A0, SWEEPS, history=True)
    t_tucker = time.time() - t0 - t_gen
    nx = oracle.sumsq(X)
    tucker_rel = oracle.tucker_rel_residual(X, G, A)
    core32 = G.astype(np.float32)
    np.save(os.path.join(HERE, "real512_core.npy"), core32)
    np.savez(os.path.join(HERE, "real512_factors.npz"), *[a.astype(np.float32) for a in A])
    B, _ = oracle.cp_ls(core32.astype(np.float64), B0, CP_SWEEPS)
    core_cp_rel = oracle.cp_rel_residual(core32, B)
    C = oracle.lift(A, B)
    cp_rel = oracle.cp_rel_residual(X, C)
    out = {"about": "FP64 oracle, real-valued CANDELINC on a 512^3 real tensor (see the docstring of "
                    "make_real512_reference.py)",
           "seed": SEED, "dims": list(dims), "planted_rank": PLANTED, "noise": NOISE, "multirank": list(ranks),
           "sweeps": SWEEPS, "cp_rank": RANK, "cp_sweeps": CP_SWEEPS,
           "tucker_rel": tucker_rel, "tucker_rel_history": [float(np.sqrt(2.0 * h / nx)) for h in hist],
           "core_npy": "real512_core.npy", "factors_npz": "real512_factors.npz",
           "core_cp_rel": core_cp_rel, "cp_rel": cp_rel,
           "congruence_with_planted": oracle.mean_congruence(C, P) if RANK <= 8 else None,
           "threads": oracle.get_threads(), "generate_seconds": t_gen, "tucker_seconds": t_tucker,
           "seconds": time.time() - t0}
    with open(os.path.join(HERE, "real512_reference.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
