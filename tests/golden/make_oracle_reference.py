"""Write oracle reference values for the full-size solver workloads.

Runs the FP64 CPU oracle (and only the oracle) on
  hg_slab_200   : 200 cells, S_8, HG g=0.9, c=0.99, tol 1e-10
  srk_slab_2000 : 2000 cells, S_64, SRK eta=1e-5, c=0.999, tol 1e-8
for source iteration, FPSA-WFD and FPSA-MPD from phi^0 = 0, and stores the
iteration counts, the first/last stopping-test values and sampled flux
moments as text.  The source-iteration solve of srk_slab_2000 takes a couple
of minutes on 8 cores, which is why its results are stored rather than
recomputed in the GPU tests.

usage: python tests/golden/make_oracle_reference.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import sn_workloads as sw  # noqa: E402

SAMPLE_CELLS = {"hg_slab_200": [0, 1, 57, 100, 198, 199],
                "srk_slab_2000": [0, 1, 2, 499, 1000, 1501, 1997, 1998, 1999]}


def main():
    out = os.path.join(HERE, "oracle_reference.txt")
    lines = ["# oracle reference values (written by make_oracle_reference.py; oracle only)",
             "# record: problem method scheme iters hist_first hist_last",
             "# sample: problem method scheme cell node l phi"]
    for prob in (sw.hg_slab_200(), sw.srk_slab_2000()):
        L = prob.L
        ls = sorted({0, 1, 2, min(5, L), L})
        for method, scheme in (("si", "wfd"), ("fpsa", "wfd"), ("fpsa", "mpd")):
            r = oracle.solve(prob, method, scheme, max_iter=200000)
            assert r["status"] == 0
            h = r["hist"]
            lines.append(f"record {prob.name} {method} {scheme} {r['iters']} {float(h[0])!r} {float(h[-1])!r}")
            for k in SAMPLE_CELLS[prob.name]:
                for nu in (0, 1):
                    for l in ls:
                        lines.append(f"sample {prob.name} {method} {scheme} {k} {nu} {l} "
                                     f"{float(r['phi'][k, nu, l])!r}")
            print(prob.name, method, scheme, r["iters"], flush=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
