"""Streaming accumulation of the steerable covariance over many images, with
checkpoint and resume (Algorithm 2, step 1, over a dataset larger than one call).

The images are produced and expanded chunk by chunk; after every chunk the FP64
accumulators {G^(k), S0, the k = 0 shift, count} and the index of the next chunk are written to a
checkpoint file (written to a temporary name, then renamed).  A run started with an
existing checkpoint of the same configuration continues after its last chunk.  The
accumulation order is fixed, so an interrupted and resumed run reproduces the
accumulators of an uninterrupted one bit for bit.

The driver only orders calls: the expansion and covariance arithmetic are the
`expand` and `accumulate` callables (by default the library's fb_expand and
fb_covariance through a Plan).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
from dataclasses import dataclass

import numpy as np


@dataclass
class StreamConfig:
    L: int
    c: float
    R: float
    n: int
    chunk: int
    seed: int
    snr: float
    precision: str

    def key(self) -> str:
        return json.dumps(self.__dict__, sort_keys=True)


class ChunkFailure(RuntimeError):
    """Raised by the failure-injection hook (tests of resume)."""


def save_checkpoint(path: str, cfg: StreamConfig, arrays: dict, count: int, next_chunk: int):
    """Write the named accumulator arrays, the image count and the next chunk index."""
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, count=np.int64(count), next_chunk=np.int64(next_chunk),
                 config=np.frombuffer(cfg.key().encode(), dtype=np.uint8),
                 **{"acc_" + k: v for k, v in arrays.items()})
    os.replace(tmp, path)


def load_checkpoint(path: str, cfg: StreamConfig):
    """(arrays, count, next_chunk) of a checkpoint written for the same configuration."""
    with np.load(path, allow_pickle=False) as z:
        key = bytes(z["config"]).decode()
        if key != cfg.key():
            raise ValueError(f"checkpoint {path} was written for another configuration: {key}")
        arrays = {k[4:]: z[k].copy() for k in z.files if k.startswith("acc_")}
        return arrays, int(z["count"]), int(z["next_chunk"])


def run_stream(cfg: StreamConfig, make_chunk, expand, accumulate, state, to_host, from_host,
               checkpoint: str | None = None, fail_at_chunk: int | None = None, log=None):
    """Process chunks [next_chunk, ceil(n / chunk)) of the configured workload.

    make_chunk(first, m) -> images of indices first .. first+m-1
    expand(images) -> coefficients;  accumulate(coeffs, state) adds them into state
    to_host(state) -> ({name: numpy array}, count);  from_host(arrays, count) -> state
    fail_at_chunk: raise ChunkFailure after expanding that chunk, before accumulating it
    Returns the state after the last chunk.
    """
    nchunks = (cfg.n + cfg.chunk - 1) // cfg.chunk
    start = 0
    if checkpoint and os.path.exists(checkpoint):
        arrays, count, start = load_checkpoint(checkpoint, cfg)
        state = from_host(arrays, count)
        if log:
            log(f"resuming at chunk {start}/{nchunks} ({count} images accumulated)")
    for ch in range(start, nchunks):
        first = ch * cfg.chunk
        m = min(cfg.chunk, cfg.n - first)
        a = expand(make_chunk(first, m))
        if fail_at_chunk is not None and ch == fail_at_chunk:
            raise ChunkFailure(f"injected failure at chunk {ch}")
        accumulate(a, state)
        if checkpoint:
            arrays, count = to_host(state)
            save_checkpoint(checkpoint, cfg, arrays, count, ch + 1)
        if log:
            log(f"chunk {ch + 1}/{nchunks} done ({first + m} images)")
    return state


def run_on_device(cfg: StreamConfig, checkpoint: str | None = None, fail_at_chunk: int | None = None, log=None,
                  batch: int = 2048):
    """The streaming run on the current HIP device through a Plan; returns (plan, CovState)."""
    import torch

    from .fb import CovState, Plan
    from .workload import synthetic_images

    plan = Plan(cfg.L, cfg.c, cfg.R)
    images = torch.empty((cfg.chunk, cfg.L, cfg.L), dtype=torch.float32, device=plan.device)
    coeffs = torch.empty((cfg.chunk, plan.p_half, 2), dtype=torch.float32, device=plan.device)

    def make_chunk(first, m):
        return synthetic_images(plan, first, m, cfg.seed, cfg.snr, out=images[:m], batch=batch)

    def expand(x):
        return plan.expand(x, precision=cfg.precision, out=coeffs[:x.shape[0]], batch=batch)

    def accumulate(a, st):
        plan.covariance(a, st, precision=cfg.precision)

    def to_host(st):
        return {"G": st.G.cpu().numpy(), "S0": st.S0.cpu().numpy(), "shift": st.shift.cpu().numpy()}, st.count

    def from_host(arrays, count):
        return CovState(G=torch.tensor(arrays["G"], device=plan.device),
                        S0=torch.tensor(arrays["S0"], device=plan.device), count=count,
                        shift=torch.tensor(arrays["shift"], device=plan.device), shift_set=True)

    st = run_stream(cfg, make_chunk, expand, accumulate, plan.new_covariance(), to_host, from_host,
                    checkpoint=checkpoint, fail_at_chunk=fail_at_chunk, log=log)
    torch.cuda.synchronize()
    return plan, st


def main(argv=None):
    ap = argparse.ArgumentParser(description="Stream a seeded synthetic workload through the expansion and "
                                             "covariance, checkpointing after every chunk; then diagonalise.")
    ap.add_argument("--L", type=int, default=360)
    ap.add_argument("--c", type=float, default=0.5)
    ap.add_argument("--R", type=float, default=None)
    ap.add_argument("--n", type=int, default=500000)
    ap.add_argument("--chunk", type=int, default=16384)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--snr", type=float, default=1 / 50)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3"])
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--out", default=None, help="write eigenvalues and eigenvectors (.npz)")
    args = ap.parse_args(argv)
    cfg = StreamConfig(L=args.L, c=args.c, R=args.R if args.R is not None else args.L / 2, n=args.n,
                       chunk=args.chunk, seed=args.seed, snr=args.snr, precision=args.precision)

    def log(msg):
        print(f"[stream] {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    plan, st = run_on_device(cfg, checkpoint=args.checkpoint, log=log)
    t1 = time.perf_counter()
    evals, evecs, C, mean = plan.eig(st)
    evals = evals.cpu().numpy()
    log(f"{st.count} images in {t1 - t0:.1f} s; largest eigenvalue {evals.max():.6g}")
    if args.out:
        np.savez(args.out, evals=evals, evecs=evecs.cpu().numpy(), mean=mean.cpu().numpy(),
                 p=plan.p, coef_off=plan.coef_off, cov_off=plan.cov_off)
    return 0


if __name__ == "__main__":
    sys.exit(main())
