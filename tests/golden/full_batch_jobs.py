"""Expected outputs of a mixed-level job list at N = 2^16, written by the oracle.

Each job (Algorithm 1 up to EvalMod, at the ciphertext's own level) is: the fused
conv (Sec. 4) with a plan encoded for the top level and applied with the first l+1
residues of its diagonals -> rescale -> exact drop to level 0 -> ModRaise ->
CoeffToSlot in three groups with lazy giant steps -> real split (Algorithm 1, up to ModEval).
The oracle computes every job; this script stores the SHA-256 of each output
ciphertext (coefficient form, uint64 little-endian, [2][l+1][N] C order) in
`full_batch_jobs.json`, so the GPU test can compare the library's batched schedule
with it word for word without re-running hours of CPU work.

Run from the repository root (calls only `oracle/` and `synth`):

    python tests/golden/full_batch_jobs.py

The job list and its inputs are defined here and imported by the GPU test: the
plans' integer diagonals, the input plaintext and the encryption randomness are the
oracle's and synth's, never the library's.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle.plans as PL  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_batch_jobs.json")
TOP = 23
# (plan name, ciphertext level, encryption sub-stream): the two "3x3b" jobs share one
# plan at different levels, so the batched schedule runs them together across levels
JOBS = [("3x3b", 9, 301), ("3x3", 11, 302), ("3x3b", 13, 303)]


def plan_weights(o):
    """conv weights of each plan: the workload's 3x3 kernel and a second seeded one"""
    C = o.C
    return {"3x3": o.K, "3x3b": synth.uniform_real((C, C, 3, 3), o.w["data_seed"], 200)}


def oracle_plans(o):
    """{name: (Bsgs, {j: integer diagonal at the top level})} of the fused conv plans"""
    out = {}
    for name, K in plan_weights(o).items():
        bs, _, _, blocks = PL.block_conv_plan(PL.taps_same(K), o.C, o.C, o.W, o.N, fuse=True)
        out[name] = (bs, PL.encode_diagonals(blocks[(0, 0)], o.N, float(o.ring.q[TOP]), o.ring, TOP))
    return out


def encrypt(o, level, sub):
    """(plaintext residues, oracle ciphertext) of the workload image at `level`"""
    m = o.ring.to_rns(o.input_plaintext(), level)
    a, e = synth.enc_randomness(o.ring.q[:level + 1], o.N, o.w["data_seed"], sub)
    return m, o.ring.encrypt_sk(level, o.s, m, a, e)


def digest(arr):
    return hashlib.sha256(np.ascontiguousarray(arr, dtype="<u8").tobytes()).hexdigest()


def run_job(o, plans, name, level, sub):
    bs, pts = plans[name]
    pts_l = {j: v[:level + 1] for j, v in pts.items()}
    _, x = encrypt(o, level, sub)
    y = o.ctx.ct_rescale(level, o.ctx.bsgs(level, x, bs, pts_l))
    return o.ctx.coeff_to_slot(y[:, :1], [p for p, _ in o.cts], [q for _, q in o.cts], lazy=True)


def main():
    from tests.oracle_workload import OracleWorkload
    t0 = time.time()
    o = OracleWorkload("full", with_cts=True, cts_split=False)  # CoeffToSlot with the default split
    plans = oracle_plans(o)
    gs = set(o.galois_elements())
    for bs, _ in plans.values():
        gs |= {PL.galois_elt(r, o.N) for r in bs.rotations()}
    o.make_keys(sorted(gs))
    rows = []
    for name, level, sub in JOBS:
        re, im = run_job(o, plans, name, level, sub)
        rows.append({"plan": name, "level": level, "sub": sub, "out_level": TOP - len(o.cts),
                     "re_sha256": digest(re), "im_sha256": digest(im)})
        print("job %s at level %d: %.1f s" % (name, level, time.time() - t0), flush=True)
    doc = {"workload": "full (N=2^16, 24+8 primes, alpha=8)", "cts_groups": len(o.cts), "lazy_cts": True,
           "plan_level": TOP, "jobs": rows,
           "command": "python tests/golden/full_batch_jobs.py (oracle only)"}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
