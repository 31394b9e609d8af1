"""The allocation-free FP64 eigensystem check (epoch_eigen_residual_noalloc) against the check
that set_epoch_eigensystems runs, through the C ABI: the same residual bits for every system, on
consecutive calls whose second and third are smaller (fewer states, fewer systems) than the
first, so the fixed scratch holds the previous call's larger contents."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1309_3075_amd import _abi
from paper_1309_3075_amd import workloads as W
from paper_1309_3075_amd.eigen import eigensystem
from paper_1309_3075_amd.likelihood import EpochLikelihood

pytestmark = pytest.mark.gpu


def _device_order(e):
    """Columns in the order set_epoch_eigensystems keeps them (complex pairs first), so that
    both checks contract over the states in the same order."""
    K = len(e.lambda_re)
    order = []
    for j in range(K):
        if e.lambda_im[j] > 0:
            order += [j, j + 1]
    order += [j for j in range(K) if e.lambda_im[j] == 0]
    return (e.V[:, order], e.Vinv[order, :], e.lambda_re[order], e.lambda_im[order])


def _systems(kind, rng):
    if kind == "codon":  # 61 states, four GY94 processes and one with a wrong eigenvalue
        pic = W.f3x4_frequencies(np.stack([rng.dirichlet(np.ones(4) * 10) for _ in range(3)]))
        Qs = [W.gy94(3.0, w, pic) for w in (0.2, 1.0, 2.5, 0.5, 0.7)]
        es = [eigensystem(Q, pic) for Q in Qs]
        es[-1].lambda_re[3] += 0.05
    elif kind == "trait":  # 40-state asymmetric rates: complex pairs
        Qs = [W.sparse_asymmetric(40, 0.2, rng) for _ in range(3)]
        es = [eigensystem(Q) for Q in Qs]
    else:  # 4 states, two HKY processes
        pi = rng.dirichlet(np.ones(4) * 5)
        Qs = [W.hky(k, pi) for k in (2.0, 8.0)]
        es = [eigensystem(Q, pi) for Q in Qs]
    return Qs, es


def _library_residuals(Qs, es):
    K, S = Qs[0].shape[0], len(Qs)
    lik = EpochLikelihood(2, 1, K, 1, S, 1, "fp64")
    out = []
    for s, (Q, e) in enumerate(zip(Qs, es)):
        out.append(lik.set_eigensystem(s, e.V, e.Vinv, e.lambda_re, e.lambda_im if e.is_complex else None, Q))
    lik.close()
    return np.array(out)


def _noalloc_residuals(Qs, es):
    lib = _abi.load()
    K, S = Qs[0].shape[0], len(Qs)
    cols = [_device_order(e) for e in es]
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    V = dev(np.stack([c[0] for c in cols]))
    Vi = dev(np.stack([c[1] for c in cols]))
    lr = dev(np.stack([c[2] for c in cols]))
    complex_ = any(e.is_complex for e in es)
    li = dev(np.stack([c[3] for c in cols])) if complex_ else None
    Q = dev(np.stack(Qs))
    res = torch.full((S,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    rc = lib.epoch_eigen_residual_noalloc(K, S, V.data_ptr(), Vi.data_ptr(), lr.data_ptr(),
                                          li.data_ptr() if li is not None else None, Q.data_ptr(),
                                          res.data_ptr(), stream.cuda_stream)
    _abi.check(rc)
    stream.synchronize()
    return res.cpu().numpy()


def test_noalloc_eigen_check_matches_set_epoch_eigensystems():
    rng = np.random.default_rng(2024)
    for kind in ("codon", "trait", "hky"):
        Qs, es = _systems(kind, rng)
        want = _library_residuals(Qs, es)
        got = _noalloc_residuals(Qs, es)
        assert np.array_equal(got, want), (kind, got, want)
        if kind == "codon":
            assert want[-1] > 1e-3 and np.all(want[:-1] < 1e-12), want
        else:
            assert np.all(want < 1e-6), (kind, want)


def test_noalloc_eigen_check_refuses_more_systems_than_its_scratch_holds():
    lib = _abi.load()
    buf = torch.zeros(64 * 64, dtype=torch.float64, device="cuda")
    p = buf.data_ptr()
    # 64 states take 48 scratch doubles per system: 2731 systems do not fit in 131072
    rc = lib.epoch_eigen_residual_noalloc(64, 2731, p, p, p, None, p, p, None)
    assert rc == _abi.EPOCH_ERR_ARG
    assert b"scratch" in lib.epoch_last_error()
    assert lib.epoch_eigen_residual_noalloc(1, 1, p, p, p, None, p, p, None) == _abi.EPOCH_ERR_ARG
