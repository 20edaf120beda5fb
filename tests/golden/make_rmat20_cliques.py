"""Writes rmat20_clique_counts.txt: the exact numbers of k-clique embeddings
(k = 3, 4, 5) of the R-MAT scale 20 bench graph (edge factor 16, a=.57
b=.19 c=.19, seed 20, symmetrised, deduplicated, loop-free).

The counts come from the oracle's clique lister alone (every k-clique listed
once at its smallest vertex of the degree orientation, times k! for the
embeddings), run on the host's cores.  The listing is exact; it takes about
15 s, 6 min and several hours on 8 cores for k = 3, 4 and 5.  Usage:
python tests/golden/make_rmat20_cliques.py [threads]
"""

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import judges  # noqa: E402

OUT = os.path.join(HERE, "rmat20_clique_counts.txt")


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    g = synth.rmat(20, 16, seed=20)
    lines = ["# exact k-clique embeddings (k! x cliques) of R-MAT scale 20 (ef 16, a=.57 b=.19 c=.19, seed 20),",
             "# symmetrised, deduplicated, loop-free; written by make_rmat20_cliques.py (oracle clique lister)",
             "# k embeddings"]
    for k in (3, 4, 5):
        t0 = time.time()
        e = judges.clique_embeddings(g, k, threads=threads)
        lines.append(f"{k} {e}")
        print(f"k={k}: {e} embeddings ({time.time() - t0:.0f} s)", flush=True)
        with open(OUT + ".tmp", "w") as f:
            f.write("\n".join(lines) + "\n")
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
