"""Write the oracle's expected values for the full-size GPU parity tests.

Calls only the CPU oracle (``oracle/``) on graphs from the seeded generators;
nothing here reads a GPU result.  Output: tests/golden/<name>.json.

    python tests/golden/make_golden.py ba1m      # BA n=1e6, m=5: scores + greedy k=10
    python tests/golden/make_golden.py rmat22    # R-MAT scale 22: scores + first greedy picks
    python tests/golden/make_golden.py ba2m      # BA n=2e6, m=8: sampled groups of the batch
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1910_13874_amd import inputs  # noqa: E402

EPS = 1e-4


def scores(g, alpha, seeds_sizes):
    out = []
    for seed, size in seeds_sizes:
        S = inputs.group(g.n, size, seed)
        t = time.time()
        c, ell, B, phi = oracle.score(g, S, alpha, EPS)
        out.append({"seed": seed, "size": size, "score": c, "ell": ell, "bound": B,
                    "phi": list(phi), "oracle_s": time.time() - t})
        print(f"  score seed={seed} |S|={size}: {c!r} ell*={ell} ({time.time() - t:.1f}s)",
              flush=True)
    return out


# the batched workload: 4,096 groups, sizes U[1,200], seed 104; sampled columns
BATCH_GROUPS, BATCH_SEED = 4096, 104
BATCH_SAMPLE = [0, 1, 17, 1000, 2047, 2048, 3333, 4095]


def batch_sample(g, alpha):
    off, mem = inputs.groups(g.n, BATCH_GROUPS, 1, 200, BATCH_SEED)
    out = []
    for j in BATCH_SAMPLE:
        S = mem[off[j]:off[j + 1]]
        t = time.time()
        c, ell, B, _ = oracle.score(g, S, alpha, EPS)
        out.append({"index": j, "size": int(S.size), "score": c, "ell": ell,
                    "oracle_s": time.time() - t})
        print(f"  group {j} |S|={S.size}: {c!r} ell*={ell} ({time.time() - t:.1f}s)", flush=True)
    return out


def main(name):
    g = inputs.workload_graph(name)
    alpha = g.default_alpha()
    rec = {"graph": name, "n": g.n, "nnz": g.nnz, "max_degree": g.max_degree, "alpha": alpha,
           "eps": EPS, "fingerprint": g.fingerprint()}
    print(f"{name}: n={g.n} nnz={g.nnz} deg_max={g.max_degree}", flush=True)
    if name == "ba1m":
        rec["scores"] = scores(g, alpha, [(102, 5), (103, 50), (104, 200), (105, 1)])
        k = 10
    elif name == "rmat22":
        rec["scores"] = scores(g, alpha, [(102, 5), (103, 100)])
        k = 3
    elif name == "ba2m":
        rec["batch"] = {"groups": BATCH_GROUPS, "seed": BATCH_SEED,
                        "sample": batch_sample(g, alpha)}
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(rec, f, indent=1)
        return
    else:
        raise SystemExit(f"unknown {name}")
    t = time.time()
    r = oracle.greedy(g, k, alpha, EPS)
    rec["greedy"] = {"k": k, "group": [int(x) for x in r["group"]],
                     "ell": [int(x) for x in r["ell"]], "L1": list(r["L1"]),
                     "U2": list(r["U2"]), "L2": list(r["L2"]), "B": list(r["B"]),
                     "evals": [int(x) for x in r["evals"]], "score": r["score"],
                     "score_ell": r["score_ell"], "oracle_s": time.time() - t}
    print(f"  greedy k={k}: {rec['greedy']['group']} ells={rec['greedy']['ell']} "
          f"({time.time() - t:.1f}s)", flush=True)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        main(nm)
