"""Write the exact ln g(E) of L x L periodic 2D Ising ferromagnets to
tests/golden/lng_L<L>.txt, for the multicanonical error metric at sizes whose
exact density of states takes minutes to compute.

The integers come from oracle.exact.exact_g (Kaufman's finite-torus partition
function evaluated modulo primes, interpolated in w = exp(4 beta J) and joined by
Chinese remaindering; the same integers Beale obtained symbolically).  Before a
file is written the script checks sum_E g(E) = 2^N, g(E) = g(-E), g(-2N) = 2
and g(-2N + 8) = 2N.  Each file holds ln g for the energy window [-2N, 0], level
k = (E + 2N)/4 = 0 .. N/2, one value per line (-inf for the empty level k = 1).

    python tests/golden/make_exact_lng.py 64 96 128 --workers 8
"""
import argparse
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402


def write(L, workers):
    N = L * L
    g = exact.exact_g(L, workers)
    assert sum(g) == 2 ** N
    assert all(g[k] == g[N - k] for k in range(N + 1))
    assert g[0] == 2 and g[2] == 2 * N and g[1] == 0
    path = os.path.join(HERE, "lng_L%d.txt" % L)
    with open(path, "w") as f:
        f.write("# exact ln g(E), %dx%d periodic Ising torus, level k = (E + 2N)/4 = 0..%d\n" % (L, L, N // 2))
        for k in range(N // 2 + 1):
            f.write("%.15g\n" % exact.big_log(g[k]) if g[k] > 0 else "-inf\n")
    print(L, path, flush=True)


if __name__ == "__main__":
    p = argparse.ArgumentParser()
    p.add_argument("L", type=int, nargs="+")
    p.add_argument("--workers", type=int, default=1)
    a = p.parse_args()
    for L in a.L:
        write(L, a.workers)
