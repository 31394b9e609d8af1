"""Host eigendecomposition of rate matrices into the library's real form.

The caller supplies eigensystems (Appendix A: one decomposition per rate
matrix, reused for every branch length and rate).  Reversible matrices with
a known stationary distribution pi use the symmetric similarity
D^1/2 Q D^-1/2 (orthogonal eigenvectors, well conditioned); any other matrix
uses a general real eigendecomposition, with complex-conjugate pairs stored
as (real part, imaginary part) columns of V.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
from scipy import linalg


@dataclass
class Eigensystem:
    V: np.ndarray          # [K][K] real form
    Vinv: np.ndarray       # [K][K]
    lambda_re: np.ndarray  # [K]
    lambda_im: np.ndarray  # [K]
    cond: float            # condition number of V

    @property
    def is_complex(self) -> bool:
        return bool(np.any(self.lambda_im != 0.0))


def eigensystem(Q: np.ndarray, pi: Optional[np.ndarray] = None) -> Eigensystem:
    Q = np.asarray(Q, dtype=np.float64)
    K = Q.shape[0]
    if pi is not None:
        pi = np.asarray(pi, dtype=np.float64)
        d = np.sqrt(pi)
        S = d[:, None] * Q / d[None, :]
        S = 0.5 * (S + S.T)
        lam, U = linalg.eigh(S)
        V = U / d[:, None]
        Vinv = U.T * d[None, :]
        return Eigensystem(V, Vinv, lam, np.zeros(K), float(np.linalg.cond(V)))
    wr, vr = linalg.eig(Q)
    lam_re = np.empty(K)
    lam_im = np.zeros(K)
    V = np.empty((K, K))
    j = 0
    while j < K:
        if wr[j].imag == 0.0:
            lam_re[j] = wr[j].real
            V[:, j] = vr[:, j].real
            j += 1
            continue
        # LAPACK returns the pair consecutively, positive imaginary part first
        a, b = wr[j].real, wr[j].imag
        if b < 0:
            a, b = wr[j + 1].real, wr[j + 1].imag
            vec = vr[:, j + 1]
        else:
            vec = vr[:, j]
        lam_re[j] = lam_re[j + 1] = a
        lam_im[j], lam_im[j + 1] = b, -b
        V[:, j] = vec.real
        V[:, j + 1] = vec.imag
        j += 2
    Vinv = np.linalg.inv(V)
    return Eigensystem(V, Vinv, lam_re, lam_im, float(np.linalg.cond(V)))
