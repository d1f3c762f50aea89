"""Write small regression fixtures from the oracle only (see README.md)."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import ntt as T  # noqa: E402
from oracle import primes as P  # noqa: E402
from oracle import ckks as CK  # noqa: E402


def main():
    q = P.prime_chain(1)[0]
    out = {}
    for log_n in (3, 4):
        n = 1 << log_n
        psi = P.psi(q, n)
        a = [(7 * i * i + 3 * i + 1) % q for i in range(n)]
        out["ntt_q%d_n%d" % (q, n)] = {"q": q, "psi": psi, "a": a,
                                       "ntt": [int(v) for v in T.ntt_def(a, q, psi)]}
    n = 16
    a = [(5 * i + 2) % q for i in range(n)]
    ah = T.ntt_def(a, q, P.psi(q, n))
    g = CK.galois_element(1, n)
    out["automorphism_g5_n16"] = {"q": q, "g": g, "ntt": [int(v) for v in ah],
                                  "rotated": [int(v) for v in CK.automorphism_ntt(ah, g)]}
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
