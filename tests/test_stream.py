"""The streaming driver (chunked accumulation with checkpoint and resume), driven on
the CPU with the FP64 oracle standing in for the library's expansion (a test fixture,
not a second backend)."""

import numpy as np
import pytest

import oracle
from paper_1412_0781_amd import synth
from paper_1412_0781_amd.stream import ChunkFailure, StreamConfig, load_checkpoint, run_stream

L, C, R = 16, 0.5, 8.0


def _setup(n=40, chunk=16):
    cfg = StreamConfig(L=L, c=C, R=R, n=n, chunk=chunk, seed=3, snr=0.1, precision="fp32")
    po = oracle.plan(L, C, R)
    p = np.array(po.p)
    cov_off = np.concatenate([[0], np.cumsum(p * p)])

    def make_chunk(first, m):
        return synth.noise_images(cfg.seed, np.arange(first, first + m), L, 1.0)

    def expand(x):
        return oracle.expand(x, po)

    def accumulate(a, st):
        for k in range(po.k_max + 1):
            o = po.coef_off[k]
            A = a[:, o:o + p[k]]
            if k == 0:
                A = A.real
            st["G"][cov_off[k]:cov_off[k + 1]] += (A.T @ np.conj(A)).real.ravel()
        st["S0"] += a[:, :p[0]].real.sum(axis=0)
        st["count"] += a.shape[0]

    def new():
        return {"G": np.zeros(cov_off[-1]), "S0": np.zeros(p[0]), "count": 0}

    def to_host(st):
        return {"G": st["G"].copy(), "S0": st["S0"].copy()}, st["count"]

    def from_host(arrays, count):
        return {"G": arrays["G"].copy(), "S0": arrays["S0"].copy(), "count": count}

    return cfg, po, (make_chunk, expand, accumulate), new, to_host, from_host


def test_stream_equals_one_shot(tmp_path):
    cfg, po, fns, new, to_host, from_host = _setup()
    st = run_stream(cfg, *fns, new(), to_host, from_host, checkpoint=str(tmp_path / "ck.npz"))
    assert st["count"] == cfg.n
    whole = new()
    fns[2](fns[1](fns[0](0, cfg.n)), whole)
    assert np.allclose(st["G"], whole["G"], rtol=1e-12, atol=1e-12 * np.abs(whole["G"]).max())
    # against the oracle's covariance blocks (Eqs.(ck),(ck_0)) from the same coefficients
    a = fns[1](fns[0](0, cfg.n))
    mean0, Cs = oracle.mean_and_covariance(a, po)
    assert np.allclose(st["S0"] / cfg.n, mean0, atol=1e-12)
    G1 = st["G"][po.p[0] ** 2:po.p[0] ** 2 + po.p[1] ** 2].reshape(po.p[1], po.p[1])
    assert np.allclose(G1 / cfg.n, Cs[1], atol=1e-12 * np.abs(Cs[1]).max())


def test_interrupted_and_resumed_is_bit_identical(tmp_path):
    cfg, po, fns, new, to_host, from_host = _setup()
    ref = run_stream(cfg, *fns, new(), to_host, from_host, checkpoint=str(tmp_path / "a.npz"))
    ck = str(tmp_path / "b.npz")
    with pytest.raises(ChunkFailure):
        run_stream(cfg, *fns, new(), to_host, from_host, checkpoint=ck, fail_at_chunk=1)
    arrays, count, nxt = load_checkpoint(ck, cfg)
    assert sorted(arrays) == ["G", "S0"]
    assert (count, nxt) == (cfg.chunk, 1)
    st = run_stream(cfg, *fns, new(), to_host, from_host, checkpoint=ck)
    assert np.array_equal(st["G"], ref["G"]) and np.array_equal(st["S0"], ref["S0"])
    assert st["count"] == ref["count"] == cfg.n


def test_checkpoint_of_another_configuration_is_refused(tmp_path):
    cfg, po, fns, new, to_host, from_host = _setup()
    ck = str(tmp_path / "c.npz")
    with pytest.raises(ChunkFailure):
        run_stream(cfg, *fns, new(), to_host, from_host, checkpoint=ck, fail_at_chunk=1)
    other = StreamConfig(**{**cfg.__dict__, "seed": cfg.seed + 1})
    with pytest.raises(ValueError):
        run_stream(other, *fns, new(), to_host, from_host, checkpoint=ck)
