"""Write full_size_samples.json: oracle values for a few trajectories of the
full-size workloads, for the sampled GPU parity tests.

The full ensembles (up to K R = 1024 trajectories of N = 50 qubits over 200
slices) are far beyond what the CPU oracle computes in a test, so a handful
of trajectories per workload is computed here once, one by one, and stored:
the overlap O_kr = <T_r|a_M> and dO_kr/du at a seeded sample of control
indices (flat order ux [M][N], uy [M][N], uzz [M][N-1]), plus the index and
value of the largest |dO| entry and the bond dimensions the trajectory
reached.  A name ending in "_self" is the self-target variant of the
workload (tests/golden/self_target.py); "_heisenberg" after the workload
name selects the paper's Heisenberg-type crosstalk.  Only `workloads` (seeded inputs) and
`oracle/` are used.

    [GOLDEN_WORKERS=n] python tests/golden/make_full_size_samples.py [workload ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import grape  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from self_target import golden_problem  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_samples.json")

# trajectories per workload: the first, the last, and two seeded ones
N_RANDOM = 2
N_ENTRIES = 48
SEED = 20260


def pick(p, rng):
    K, R = p.K, p.R
    ts = {0, K * R - 1}
    while len(ts) < 2 + N_RANDOM:
        ts.add(int(rng.integers(0, K * R)))
    return sorted(ts)


def _one(args):
    name, k, r = args
    p, _ = golden_problem(name)
    t0 = time.perf_counter()
    st = []
    O, dux, duy, duzz = grape.trajectory(p, k, r, stats=st)
    flat = np.concatenate([dux.ravel(), duy.ravel(), duzz.ravel()])
    return O, flat, int(max(s["k"] for s in st)), time.perf_counter() - t0


def sample(name, workers=1):
    p, base = golden_problem(name)
    rng = np.random.default_rng([SEED, sum(map(ord, name))])
    nctrl = 2 * p.M * p.N + p.M * (p.N - 1)
    ts = pick(p, rng)
    jobs = [(name,) + divmod(t, p.R) for t in ts]
    if workers > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(workers) as ex:
            results = list(ex.map(_one, jobs))
    else:
        results = [_one(j) for j in jobs]
    out = []
    for (_, k, r), (O, flat, dmax, secs) in zip(jobs, results):
        assert flat.size == nctrl
        idx = np.sort(rng.choice(nctrl, size=N_ENTRIES, replace=False))
        imax = int(np.argmax(np.abs(flat)))
        out.append({
            "k": k, "r": r,
            "O": [O.real, O.imag],
            "idx": [int(i) for i in idx],
            "dO": [[flat[i].real, flat[i].imag] for i in idx],
            "dO_argmax": imax,
            "dO_max": [flat[imax].real, flat[imax].imag],
            "dO_inf": float(np.max(np.abs(flat))),
            "max_bond_dim": dmax,
        })
        print(f"{name} (k={k}, r={r}): |O|={abs(O):.3e} |dO|_inf={out[-1]['dO_inf']:.3e} "
              f"max D={dmax} {secs:.1f} s", flush=True)
    cfg = dict(W.CONFIGS[base], self_target=name.endswith("_self"), xt_model=p.xt_model)
    return {"config": cfg, "nctrl": nctrl, "trajectories": out}


def main():
    names = sys.argv[1:] or ["xgate_n50", "cnot_n50", "cnot_n50_self"]
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["_about"] = ("Oracle values (tests/golden/make_full_size_samples.py) for sampled "
                      "trajectories of the full-size workloads; controls index order ux, uy, uzz.")
    workers = int(os.environ.get("GOLDEN_WORKERS", "1"))
    for name in names:
        data[name] = sample(name, workers)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
