"""50-digit mpmath evaluation of the Fisher vector for tiny inputs (test infrastructure only).

Same definition as ``fv_oracle.c`` (Algorithm 1 of the paper plus the improved-FV
normalisation), written independently in pure Python at high precision.  It bounds the
rounding error of the double-precision oracle; it is not, by itself, a check of the
definition (the closed forms, library cross-checks and invariances in the tests are).
"""
from __future__ import annotations

import mpmath as mp


def encode(X, w, mu, var, power: bool = True, l2: bool = True, dps: int = 50):
    with mp.workdps(dps):
        N = len(X)
        K = len(w)
        D = len(mu[0])
        Xm = [[mp.mpf(float(v)) for v in row] for row in X]
        wm = [mp.mpf(float(v)) for v in w]
        mum = [[mp.mpf(float(v)) for v in row] for row in mu]
        vm = [[mp.mpf(float(v)) for v in row] for row in var]
        U = [[mp.mpf(0)] * D for _ in range(K)]
        V = [[mp.mpf(0)] * D for _ in range(K)]
        for t in range(N):
            logp = []
            for k in range(K):
                q = mp.mpf(0)
                ld = mp.mpf(0)
                for d in range(D):
                    q += (Xm[t][d] - mum[k][d]) ** 2 / vm[k][d]
                    ld += mp.log(vm[k][d])
                logp.append(mp.log(wm[k]) - ld / 2 - q / 2)
            m = max(logp)
            e = [mp.exp(v - m) for v in logp]
            Z = mp.fsum(e)
            for k in range(K):
                g = e[k] / Z
                for d in range(D):
                    z = (Xm[t][d] - mum[k][d]) / mp.sqrt(vm[k][d])
                    U[k][d] += g * z
                    V[k][d] += g * (z * z - 1)
        phi = []
        for k in range(K):
            phi += [U[k][d] / (N * mp.sqrt(wm[k])) for d in range(D)]
        for k in range(K):
            phi += [V[k][d] / (N * mp.sqrt(2 * wm[k])) for d in range(D)]
        if power:
            phi = [mp.sign(p) * mp.sqrt(abs(p)) for p in phi]
        if l2:
            n = mp.sqrt(mp.fsum([p * p for p in phi]))
            if n > 0:
                phi = [p / n for p in phi]
        return [float(p) for p in phi]
