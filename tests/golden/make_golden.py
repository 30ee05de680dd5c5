"""Writes tests/golden/rmat_counts.json: exact counts on the RMAT workloads,
computed by the CPU oracle only (oracle/ + graphgen/), never by the device
path.  Run: python tests/golden/make_golden.py [--scales 18 20]

Workloads (seeded, synthetic):
  rmat18: RMAT scale 18, 16 * 2^18 distinct edges, (a,b,c,d) = (.57,.19,.19,.05), seed 18
  rmat20: RMAT scale 20, 16 * 2^20 distinct edges, same parameters, seed 20
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle    # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat_counts.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scales", type=int, nargs="+", default=[18, 20])
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for s in args.scales:
        key = f"rmat{s}"
        g = graphgen.rmat(s, seed=s)
        off, adj = oracle.canonical_csr(g.n, g.u, g.v)
        rec = data.get(key, {})
        rec.update({"scale": s, "seed": s, "edge_factor": 16, "n": g.n,
                    "input_edges": g.num_input_edges, "m": int(adj.shape[0] // 2)})
        for k in (3, 4, 5):
            if f"clique{k}" in rec:
                continue
            t = time.time()
            rec[f"clique{k}"] = oracle.clique_count(off, adj, k, args.threads)
            print(f"{key} clique{k} = {rec[f'clique{k}']} ({time.time() - t:.1f} s)", flush=True)
            data[key] = rec
            with open(OUT, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
        if s <= 18:
            if "motif4" not in rec:
                rec["motif3"] = oracle.motif3(off, adj, args.threads)
                rec["motif4"] = oracle.motif4(off, adj, args.threads)
            for name, fn in (("diamond", oracle.list_diamonds), ("4-cycle", oracle.list_c4)):
                if f"sl_{name}" in rec:
                    continue
                t = time.time()
                total, chk, _ = fn(off, adj, 0, args.threads)
                rec[f"sl_{name}"] = {"total": total, "checksum": chk}
                print(f"{key} {name} {total} {chk} ({time.time() - t:.1f} s)", flush=True)
        data[key] = rec
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
