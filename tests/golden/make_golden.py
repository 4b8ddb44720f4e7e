"""Writes brute_small.json: dense 2^n brute-force estimates for a few seeded
walker/shadow pairs at n = 3, 4, 5 (inputs stored alongside).  Calls only the
oracle's brute force.  Run:  python tests/golden/make_golden.py"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import brute  # noqa: E402


def haar_so(rng, d):
    Qm, R = np.linalg.qr(rng.standard_normal((d, d)))
    Qm = Qm * np.sign(np.diag(R))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] *= -1
    return Qm


def main():
    rng = np.random.default_rng(20250627)
    cases = []
    for (n, eta, orth) in [(3, 2, True), (4, 2, True), (4, 4, False), (5, 2, True), (5, 4, False)]:
        Z = rng.standard_normal((n, eta)) + 1j * rng.standard_normal((n, eta))
        phi = np.linalg.qr(Z)[0] if orth else Z
        Q = haar_so(rng, 2 * n)
        b = rng.integers(0, 2, n - 1)
        bits = int(sum(int(v) << j for j, v in enumerate(b)) | ((int(b.sum()) % 2) << (n - 1)))
        o = brute.overlap_pair(phi, Q, bits)
        cases.append(dict(n=n, eta=eta, phi_re=phi.real.tolist(), phi_im=phi.imag.tolist(),
                          Q=Q.tolist(), bits=bits, o=[o.real, o.imag]))
    with open(os.path.join(HERE, "brute_small.json"), "w") as f:
        json.dump(dict(source="oracle.brute (dense 2^n plain definition, o = 2<0|rho_hat|phi>)",
                       cases=cases), f, indent=1)


if __name__ == "__main__":
    main()
