"""Write tests/golden/dense_n<n>_optimum.json from the CPU oracle alone.

The dense symmetric instance of size n (F, D ~ U{0..99}, zero diagonals,
seed 0; n = 14 by default) is solved by two independent exact solvers of the
oracle -- the RLT2 dual-ascent B&B and the Gilmore-Lawler-bounded B&B -- and
the file is written only when they agree.
Run:  python tests/golden/make_golden.py [n]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1710_03732_amd import instances as I  # noqa: E402


def main(n: int = 14):
    inst = I.dense_instance(n, 0)
    F, D, B = inst.arrays()
    t0 = time.time()
    r_obj, r_perm, r_st = O.bnb(F, D, B, node_iters=100, window=25, min_improve=2e-4)
    t1 = time.time()
    g_obj, g_perm, g_nodes = O.glb_bnb(F, D, B)
    t2 = time.time()
    if r_obj != g_obj:
        raise SystemExit(f"exact solvers disagree: {r_obj} vs {g_obj}")
    out = {
        "instance": f"dense symmetric n={n}, F and D ~ U{{0..99}}, zero diagonals, seed 0",
        "n": n,
        "optimum": r_obj,
        "perm": [int(x) for x in r_perm],
        "rlt2_bnb_optimum": r_obj,
        "rlt2_bnb_stats": {k: int(v) for k, v in r_st.items()},
        "rlt2_bnb_seconds": round(t1 - t0, 1),
        "glb_bnb_optimum": g_obj,
        "glb_bnb_nodes": int(g_nodes),
        "glb_bnb_seconds": round(t2 - t1, 1),
        "written_by": "tests/golden/make_golden.py (CPU oracle only)",
    }
    with open(os.path.join(HERE, f"dense_n{n}_optimum.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 14)
