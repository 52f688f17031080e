#!/usr/bin/env python3
"""Throughput of the Fourier-Bessel expansion + steerable covariance on one MI355X.

Default workload (the headline configuration, --workload c3): n = 100 000 synthetic
cryo-EM-shaped images, L = 256, support radius R = 128, band limit c = 1/2.  Each image is
the synthesis T a of random Fourier-Bessel coefficients with variance (1+q)^-2 (1+|k|)^-1
plus white Gaussian noise at SNR 1/20, generated on the device from seed 0
(Philox-4x32-10) before timing starts; inputs are resident in HBM when the timed region
starts.

One step = the whole hot path over all n images: fb_expand (polar NUFFT, angular FFT,
radial quadrature) then fb_covariance (G^(k) += Re(A A^*), k = 0 sums).  Both arithmetic
forms are timed, FP32 and split-BF16x3; `value` is the BF16x3 form.  The plan (tables) and
the eigendecomposition are outside the timed region (the eigendecomposition is timed on
its own and reported).

Other workloads (not the headline line):
  --workload c2  n = 100 000, L = 128, R = 64, SNR 1/20, resident; value = the FP32 form
  --workload c4  differentiation: n = 20 000, L = 128, forward expansion, fixed Wiener-like
                 shrinkage, adjoint synthesis and the backward pass of both (autograd);
                 value = images/s of forward + backward, FP32
  --workload c5  L = 360, R = 180, SNR 1/50, images generated on the device chunk by chunk
                 (16 384 per chunk) and the covariance accumulated across chunks; value =
                 images/s of expansion + covariance (generation untimed).  --n sets the
                 images streamed (default two chunks; 500 000 is the whole set)

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "images/s (FB coeffs + covariance) at L=256, BF16x3 vs FP32, ≤1e-5 rel err"
HBM_PEAK_GBS = 8000.0
# Published MI355X peaks: FP32 vector (and FP32 matrix) 157.3 TFLOP/s, dense BF16 matrix
# 2.5 PFLOP/s.  The library emits no packed (two-wide) FP32 instructions, so its vector
# FP32 code can issue at most half the published rate: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flop x 2.4 GHz = 78.6 TFLOP/s, reported beside the published-peak fraction.
FP32_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
ALU_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# LDS read rate of ds_read_b128 measured on the device (a plain read loop): the practical
# limit of the gather, whose every tap is one 16-byte LDS read per lane
LDS_MEASURED_TBS = 116.0
PROFILES = os.path.join(ROOT, "profiles")

# workload -> defaults (kind: resident = all images in HBM, stream = generated chunk by
# chunk, autograd = forward + backward of the differentiation workload)
WORKLOADS = {
    "c3": {"L": 256, "n": 100000, "snr": 1 / 20, "cpu_sample": 8, "head": "bf16x3", "kind": "resident",
           "forms": "fp32,bf16x3", "dict_images": 2000, "dict_pixels": 128},
    "c2": {"L": 128, "n": 100000, "snr": 1 / 20, "cpu_sample": 48, "head": "fp32", "kind": "resident",
           "forms": "fp32,bf16x3", "dict_images": 2000, "dict_pixels": 128},
    "c4": {"L": 128, "n": 20000, "snr": 1 / 20, "cpu_sample": 16, "head": "fp32", "kind": "autograd",
           "forms": "fp32", "dict_images": 0, "dict_pixels": 0},
    "c5": {"L": 360, "n": 2 * 16384, "snr": 1 / 50, "cpu_sample": 4, "head": "bf16x3", "kind": "stream",
           "forms": "fp32,bf16x3", "dict_images": 1000, "dict_pixels": 64, "chunk": 16384},
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_per_image(plan) -> dict:
    """Minimum HBM bytes each kernel must move per image (read its input once, write its output once)."""
    L, N, M2 = plan.L, plan.grid_n, plan.grid_n // 2 + 2 * (plan.kernel_w // 2 + 1) + 1
    H = plan.n_theta // 2
    c8 = 8
    img = 4 * L * L
    g1 = c8 * M2 * L
    g = c8 * M2 * N
    P = c8 * plan.n_xi * H
    fh = c8 * (plan.k_max + 1) * plan.n_xi
    co = c8 * plan.p_half
    y = c8 * (N // 2 + 1) * N        # folded half-plane grid of the adjoint
    y1 = c8 * (N // 2 + 1) * L       # adjoint column-pass output
    return {
        "fwd_rows": img + g1,
        "fwd_cols": g1 + g,
        "fwd_gather": g + P,
        "fwd_angular": P + fh,
        "radial_fwd": fh + co,
        "covariance": co,
        "radial_adj": co + fh,
        "adj_angular": fh + P,
        "adj_spread": P + y,
        "adj_cols": y + y1,
        "adj_rows": y1 + img,
    }


def algorithmic_flops_per_image(plan) -> dict:
    """Textbook flops per image of each stage (the counts of the method's work, not of this
    implementation's instructions):
      2-D FFT of the N x N oversampled grid   2.5 N^2 log2(N^2)   (shared by rows and columns
                                                                   in proportion to their transforms)
      interpolation (gather, spread)          4 w^2 per polar node of the half rings
      angular FFT                             5 H log2 H per ring (complex FFT of length H = n_theta/2)
      radial quadrature Eq.(a), its transpose 4 n_xi sum_{k>0} p_k + 2 n_xi p_0
      covariance Eq.(ck)                      4 sum_k p_k^2"""
    W, N, H = plan.kernel_w, plan.grid_n, plan.n_theta // 2
    M2 = N // 2 + 2 * (W // 2 + 1) + 1
    fft2 = 2.5 * N * N * math.log2(N * N)
    rows_share = (plan.L / 2) / (plan.L / 2 + M2)  # row-pair transforms vs column transforms
    p = [int(x) for x in plan.p]
    radial = 4 * plan.n_xi * sum(p[1:]) + 2 * plan.n_xi * p[0]
    ang = plan.n_xi * 5 * H * math.log2(H)
    gather = 4 * W * W * plan.n_xi * H
    return {
        "fwd_rows": fft2 * rows_share,
        "fwd_cols": fft2 * (1 - rows_share),
        "fwd_gather": gather,
        "fwd_angular": ang,
        "radial_fwd": radial,
        "covariance": 4 * sum(x * x for x in p),
        "radial_adj": radial,
        "adj_angular": ang,
        "adj_spread": gather,
        "adj_cols": fft2 * (1 - rows_share),
        "adj_rows": fft2 * rows_share,
    }


def stage_peak_tflops(stage: str, precision: str) -> float:
    """Peak of the unit that does a stage's arithmetic: the matrix cores for the two
    contractions (BF16 at three products per FP32 product in the BF16x3 form), the FP32
    vector units otherwise."""
    if stage in ("radial_fwd", "covariance") and precision == "bf16x3":
        return BF16_MFMA_PEAK_TFLOPS / 3.0
    return FP32_PEAK_TFLOPS


def step_roofline(plan, precision: str, stages: dict, images: int, step_ms: float, n: int,
                  passes: int = 1) -> dict:
    """Whole-step roofline: sum over the step's stages of max(bytes / HBM peak, flops / peak)
    per image, divided by the measured time per image; also each stage's own fraction (its
    bound over its measured average time per image) and the bound of a fully fused path,
    which moves only the image and its coefficients through HBM.  `images` = images over all
    timed steps, n = images per step, `passes` = times each image runs through every stage in
    one step (2 for forward + backward of the differentiation workload, whose backward pass
    applies the adjoint of each transform: T for T* and T* for T)."""
    bpi = algorithmic_bytes_per_image(plan)
    fpi = algorithmic_flops_per_image(plan)
    bound = 0.0
    per_stage = {}
    present = [st for st in bpi if st in stages and stages[st]["launches"]]
    for st in present:
        t = max(bpi[st] / (HBM_PEAK_GBS * 1e9), fpi[st] / (stage_peak_tflops(st, precision) * 1e12))
        bound += passes * t
        per_stage[st] = round(t / (stages[st]["total_ms"] * 1e-3 / (images * passes)), 4)
    measured = step_ms * 1e-3 / n
    # image in, coefficients out (expansion) and back (synthesis), per pass
    directions = sum(1 for pre in ("fwd_", "adj_") if any(st.startswith(pre) for st in present))
    irreducible = passes * directions * (4 * plan.L * plan.L + 8 * plan.p_half)
    fused = max(irreducible / (HBM_PEAK_GBS * 1e9),
                passes * sum(fpi[st] / (stage_peak_tflops(st, precision) * 1e12) for st in present))
    return {"bound_us_per_image": round(bound * 1e6, 4), "measured_us_per_image": round(measured * 1e6, 4),
            "frac": round(bound / measured, 4), "fused_bound_us_per_image": round(fused * 1e6, 4),
            "fused_frac": round(fused / measured, 4), "stage_frac": per_stage,
            "mflop_per_image": round(passes * sum(fpi[st] for st in present) / 1e6, 2),
            "unfused_MB_per_image": round(passes * sum(bpi[st] for st in present) / 1e6, 3),
            "irreducible_MB_per_image": round(irreducible / 1e6, 3)}


def kernel_roofline(plan, stages: dict, images: int, precision: str) -> dict:
    """The dominant kernel (largest total time among the stages with known algorithmic bytes)
    against its roofline: HBM when its arithmetic intensity is below the ridge point of its
    unit, else that unit's peak.  achieved = algorithmic bytes (or flops) of one launch over
    the average launch duration measured with HIP events on the launch stream.  `images` =
    images the timed region ran through each stage (all of its launches together)."""
    bpi = algorithmic_bytes_per_image(plan)
    fpi = algorithmic_flops_per_image(plan)
    dom = max((s for s in stages if s in bpi), key=lambda s: stages[s]["total_ms"])
    per_launch_images = images / stages[dom]["launches"]
    sec = stages[dom]["avg_ms"] * 1e-3
    alg_bytes = bpi[dom] * per_launch_images
    hbm_achieved = alg_bytes / sec / 1e9
    tpi = stored_traffic_per_image(dom, plan.L)
    traffic = round(tpi * per_launch_images) if tpi is not None else None
    flops = fpi.get(dom, 0) * per_launch_images
    peak = stage_peak_tflops(dom, precision)
    mfma = dom in ("radial_fwd", "covariance", "radial_adj")
    if flops / alg_bytes > (peak * 1e12) / (HBM_PEAK_GBS * 1e9):
        ach = flops / sec / 1e12
        roofline = {"bound": "mfma" if mfma else "alu", "kernel": dom, "achieved": round(ach, 2),
                    "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4), "traffic": traffic,
                    "flops_per_launch": int(flops), "hbm_algorithmic_GBps": round(hbm_achieved, 1),
                    "hbm_frac": round(hbm_achieved / HBM_PEAK_GBS, 4)}
        if not mfma:
            roofline["frac_of_nonpacked_fp32_issue_rate"] = round(ach / ALU_FP32_NONPACKED_TFLOPS, 4)
    else:
        # arithmetic intensity below the ridge point: the attainable rate is set by HBM
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(hbm_achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(hbm_achieved / HBM_PEAK_GBS, 4), "traffic": traffic}
        if flops:
            ach = flops / sec / 1e12
            roofline.update({"flops_per_launch": int(flops), "flop_rate_TFLOPs": round(ach, 2),
                             "flop_frac_of_published_peak": round(ach / peak, 4)})
            if not mfma:
                roofline["frac_of_nonpacked_fp32_issue_rate"] = round(ach / ALU_FP32_NONPACKED_TFLOPS, 4)
    if dom in ("fwd_gather", "adj_spread"):
        # w x w taps per node and image pair, one 16-byte LDS read each (8 bytes per image)
        lds = plan.kernel_w ** 2 * 8 * plan.n_xi * (plan.n_theta // 2) * per_launch_images
        roofline["lds_read_TBs"] = round(lds / sec / 1e12, 1)
        roofline["lds_frac_of_measured"] = round(lds / sec / 1e12 / LDS_MEASURED_TBS, 4)
    roofline.update({"bytes_per_launch": int(alg_bytes), "images_per_launch": round(per_launch_images, 1),
                     "avg_launch_ms": round(stages[dom]["avg_ms"], 4)})
    return roofline


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def stored_traffic_per_image(stage: str, L: int):
    """HBM bytes per image of `stage` from the committed counter summary (rocprofv3 FETCH_SIZE /
    WRITE_SIZE, scaled by the plain-copy calibration), or None if the kernel sources changed
    since the counters were taken."""
    path = os.path.join(PROFILES, f"{stage}_hbm_counters_L{L}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    from paper_1412_0781_amd.prof_summary import source_digest
    if kv.get("source_digest") != source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_image"])
    except (KeyError, ValueError):
        return None


def make_images(plan, n, seed, snr, chunk=4096):
    import torch

    from paper_1412_0781_amd.workload import noise_sigma, synthetic_images

    images = torch.empty((n, plan.L, plan.L), dtype=torch.float32, device=plan.device)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        synthetic_images(plan, s, m, seed, snr, out=images[s:s + m])
    torch.cuda.synchronize()
    return images, noise_sigma(plan, snr)


def _stage_totals(prof: dict) -> dict:
    return {name: {"total_ms": ms, "launches": cnt, "avg_ms": ms / max(cnt, 1)} for name, (ms, cnt) in prof.items()}


def time_form(plan, images, coeffs, precision, steps, warmup, pass_images):
    """`steps` timed steps of expansion + covariance over all resident images."""
    import torch

    st = plan.new_covariance()
    stream = torch.cuda.current_stream()

    def step():
        st.G.zero_()
        st.S0.zero_()
        st.count = 0
        st.shift_set = False  # each step takes the shift from its first images again
        plan.expand(images, precision=precision, out=coeffs, batch=pass_images)
        plan.covariance(coeffs, st, precision=precision)

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"{precision}: warmup step {i + 1}/{warmup} done")
    plan.profile_read(reset=True)
    plan.profile(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.profile(False)
    prof = plan.profile_read(reset=True)
    ev_ms = e0.elapsed_time(e1)
    log(f"{precision}: {steps} steps in {wall:.3f} s (events {ev_ms / 1e3:.3f} s)")
    return wall, ev_ms, prof, st


def time_stream(plan, n, chunk, seed, snr, precision, pass_images, warmup=1):
    """Images generated on the device chunk by chunk (untimed), each chunk expanded and added to
    one covariance accumulator (timed with HIP events); `warmup` chunks first, not counted.
    Returns (timed ms, chunks timed, per-kernel profile, covariance state)."""
    import torch

    from paper_1412_0781_amd.workload import synthetic_images

    images = torch.empty((chunk, plan.L, plan.L), dtype=torch.float32, device=plan.device)
    coeffs = torch.empty((chunk, plan.p_half, 2), dtype=torch.float32, device=plan.device)
    stream = torch.cuda.current_stream()
    for w in range(warmup):
        synthetic_images(plan, 0, chunk, seed, snr, out=images)
        plan.covariance(plan.expand(images, precision=precision, out=coeffs, batch=pass_images),
                        precision=precision)
        torch.cuda.synchronize()
        log(f"{precision}: warm-up chunk {w + 1}/{warmup} done")
    st = plan.new_covariance()
    plan.profile_read(reset=True)
    total_ms = 0.0
    nch = (n + chunk - 1) // chunk
    for ch in range(nch):
        first = ch * chunk
        m = min(chunk, n - first)
        synthetic_images(plan, first, m, seed, snr, out=images[:m])
        torch.cuda.synchronize()
        plan.profile(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.expand(images[:m], precision=precision, out=coeffs[:m], batch=pass_images)
        plan.covariance(coeffs[:m], st, precision=precision)
        e1.record(stream)
        torch.cuda.synchronize()
        plan.profile(False)
        total_ms += e0.elapsed_time(e1)
        log(f"{precision}: chunk {ch + 1}/{nch} ({first + m} images) done")
    prof = plan.profile_read(reset=True)
    return total_ms, nch, prof, st


def time_autograd(plan, n, seed, snr, steps, warmup, pass_images):
    """The differentiation workload: I -> a = T* I (FBExpand) -> h . a with the fixed Wiener-like
    shrinkage h = v / (v + sigma^2) -> T(h . a) (FBSynth) -> loss = ||T(h . a) - I_clean||^2, and
    the backward pass to dloss/dI; `steps` timed forward + backward steps over all n images."""
    import numpy as np
    import torch

    from paper_1412_0781_amd import fb_expand, fb_synth, synth
    from paper_1412_0781_amd.fb import synth_normals
    from paper_1412_0781_amd.workload import coefficient_scale, noise_sigma

    L = plan.L
    a = synth_normals(seed, synth.STREAM_COEF, 0, n, 2 * plan.p_half, 1.0, plan.device).view(n, plan.p_half, 2)
    a.mul_(coefficient_scale(plan))
    clean = plan.adjoint(a, batch=pass_images)
    del a
    sig = noise_sigma(plan, snr)
    noisy = clean + synth_normals(seed, synth.STREAM_NOISE, 0, n, L * L, sig, plan.device).view(n, L, L)
    v = synth.coef_variance(plan.k.astype(np.float64), plan.q.astype(np.float64))
    h = torch.tensor((v / (v + sig * sig)).astype(np.float32), device=plan.device)[None, :, None]
    x = noisy.detach().requires_grad_(True)
    torch.cuda.synchronize()

    def step():
        x.grad = None
        rec = fb_synth(fb_expand(x, plan) * h, plan)
        loss = ((rec - clean) ** 2).sum()
        loss.backward()
        return loss

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"autograd: warmup step {i + 1}/{warmup} done")
    plan.profile_read(reset=True)
    plan.profile(True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.profile(False)
    prof = plan.profile_read(reset=True)
    log(f"autograd: {steps} steps in {wall:.3f} s")
    return wall, e0.elapsed_time(e1), prof, sig


def cpu_baseline(plan_args, sample, seed, snr, kind):
    """The FP64 oracle, timed on the host on a bounded sample of the same workload: expansion +
    covariance, or for the differentiation workload the forward expansion, shrinkage and synthesis
    and the backward pass (two expansions and two syntheses per image)."""
    import numpy as np

    import oracle
    from paper_1412_0781_amd import synth

    L, c, R = plan_args
    po = oracle.plan(L, c, R)
    idx = np.arange(sample)
    kk, qq = po.kq[:, 0], po.kq[:, 1]
    a = synth.random_coefficients(seed, idx, kk, qq)
    sigma = math.sqrt(synth.noise_sigma2(kk, qq, L, snr))
    img = np.empty((sample, L, L), np.float32)
    clean = np.empty((sample, L, L))
    noise = synth.noise_images(seed, idx, L, sigma)
    for i in range(sample):
        clean[i] = oracle.adjoint(a[i:i + 1], po)[0]
        img[i] = (clean[i] + noise[i]).astype(np.float32)
        log(f"cpu baseline: synthesised sample image {i + 1}/{sample} on the host (not timed)")
    _ = po.B  # radial table: part of the plan, outside the timed region
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = len(os.sched_getaffinity(0))
    log(f"cpu baseline: timing the oracle on {sample} images with {cores} BLAS threads")
    t0 = time.perf_counter()
    coef = np.empty((sample, po.p_half), np.complex128)
    if kind == "autograd":
        v = synth.coef_variance(kk, qq)
        h = v / (v + sigma * sigma)
        w = np.where(kk > 0, 2.0, 1.0)
        for i in range(sample):
            x = img[i:i + 1].astype(np.float64)
            coef[i] = oracle.expand(x, po)[0]
            rec = oracle.adjoint(h * coef[i:i + 1], po)
            g = 2.0 * (rec - clean[i:i + 1])
            gb = w * oracle.expand(g, po)               # gradient of the synthesis
            _ = oracle.adjoint(h * gb / w, po)          # transpose of the expansion (weight 1)
            log(f"cpu baseline: oracle forward + backward of image {i + 1}/{sample} done")
        what = "forward expansion, shrinkage, synthesis and the backward pass in FP64"
    else:
        for i in range(sample):
            coef[i] = oracle.expand(img[i:i + 1].astype(np.float64), po)[0]
            log(f"cpu baseline: oracle expansion of image {i + 1}/{sample} done")
        oracle.mean_and_covariance(coef, po)
        what = "expansion + covariance in FP64"
    dt = time.perf_counter() - t0
    return img, coef, po, {"value": sample / dt, "unit": "images/s", "cores": int(cores), "kind": "oracle",
                           "cpu": cpu_model(),
                           "sample": f"{sample} images of the same workload (L={L}, R={R}, c={c}), {what}, "
                                     f"{dt:.1f} s (bounded to about half a minute of host time)"}


def dictionary_accuracy(plan, po, n, D, precisions, seed=21, offset=3.0):
    """Error of every result against the FP64 oracle at the benchmark's shape: n images that
    combine D random pixels with values N(offset, 1) (a dominant mean image), whose oracle
    coefficients are the same combination of the oracle expansions of the D single-pixel
    images; coefficients (whole and worst k block), C^(k) (relative Frobenius, max over k),
    the eigenvalues (per block, relative to the block's largest) and the k = 0 mean."""
    import numpy as np
    import torch

    import oracle

    rng = np.random.default_rng(seed)
    L = po.L
    flat = rng.choice(L * L, size=D, replace=False)
    rows, cols = flat // L, flat % L
    V = (rng.standard_normal((n, D)) + offset).astype(np.float32)
    log(f"accuracy: oracle expansion of {D} single-pixel images (L={L}) on the host")
    a_ref = oracle.expand_pixel_combinations(V.astype(np.float64), rows, cols, po)
    mean_ref, C_ref = oracle.mean_and_covariance(a_ref, po)
    lam_ref, _ = oracle.eig_blocks(C_ref)
    dense = np.zeros((n, L, L), np.float32)
    dense[:, rows, cols] = V
    x = torch.tensor(dense, device=plan.device)
    out = {}
    off = po.coef_off
    for prec in precisions:
        a = plan.expand(x, precision=prec)
        st = plan.covariance(a, precision=prec)
        evals, _, C, mean = plan.eig(st)
        torch.cuda.synchronize()
        g = a.cpu().numpy().astype(np.float64)
        g = g[..., 0] + 1j * g[..., 1]
        blk = max(np.linalg.norm(g[:, off[k]:off[k + 1]] - a_ref[:, off[k]:off[k + 1]])
                  / np.linalg.norm(a_ref[:, off[k]:off[k + 1]]) for k in range(po.k_max + 1))
        Cb = plan.blocks(C.cpu().numpy())
        eC = max(np.linalg.norm(Cb[k] - C_ref[k]) / np.linalg.norm(C_ref[k]) for k in range(po.k_max + 1))
        ev = evals.cpu().numpy()
        el = max(np.max(np.abs(ev[off[k]:off[k + 1]] - lam_ref[k])) / lam_ref[k][0] for k in range(po.k_max + 1))
        out[prec] = {"coeff_rel_l2": float(np.linalg.norm(g - a_ref) / np.linalg.norm(a_ref)),
                     "coeff_worst_k_block": float(blk), "cov_max_over_k": float(eC), "eigenvalue_max": float(el),
                     "mean_rel_l2": float(np.linalg.norm(mean.cpu().numpy() - mean_ref) / np.linalg.norm(mean_ref)),
                     "sample": f"{n} images combining {D} pixels, values N({offset:g}, 1)"}
    return out


def extra_legs(plan, coeffs, evals, evecs, mean, n, sigma, pass_images):
    """Figures outside images/s at the headline shape: the SVD route, the steerable-PCA back end
    with the real-space eigenimages, the adjoint synthesis and the R / c estimate."""
    import torch

    L = plan.L

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(torch.cuda.current_stream())
        r = fn()
        e1.record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1)

    # principal components by the SVD of the coefficient matrices (Sec. III-C): the same
    # eigenvalues without forming C^(k)
    svd_ws = torch.empty(plan.svd_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    plan.svd(coeffs[:64], ws=svd_ws)  # warm-up
    torch.cuda.synchronize()
    ts = time.perf_counter()
    sv_evals, _, _ = plan.svd(coeffs, ws=svd_ws)
    torch.cuda.synchronize()
    svd_ms = 1e3 * (time.perf_counter() - ts)
    del svd_ws
    lam = evals.cpu().tolist()
    d = (sv_evals - evals).abs().cpu().tolist()
    rel = max(d[i] / max(lam[int(plan.coef_off[k])], 1e-300)
              for k in range(plan.k_max + 1) for i in range(int(plan.coef_off[k]), int(plan.coef_off[k + 1])))
    svd = {"images": n, "ms": round(svd_ms, 3), "max_eval_diff_vs_eig": rel}
    log(f"svd route: {svd}")

    # steerable-PCA back end: selection with the workload's noise variance, sPCA coefficients
    # of every image, filtered reconstruction of their FB coefficients
    n_sel, w = plan.spca_select(evals, n, sigma * sigma)
    plan.spca_coeffs(coeffs[:64], evecs, mean)  # warm-up
    cs, c_ms = timed(lambda: plan.spca_coeffs(coeffs, evecs, mean))
    _, r_ms = timed(lambda: plan.spca_reconstruct(cs, evecs, mean, w))
    del cs
    spca_bytes = 2 * 8 * plan.p_half * n
    spca = {"selected_components": int(n_sel.sum().item()), "coeffs_ms": round(c_ms, 3),
            "reconstruct_ms": round(r_ms, 3), "coeffs_images_per_s": round(n / (c_ms * 1e-3), 1),
            "coeffs_hbm_GBps": round(spca_bytes / (c_ms * 1e-3) / 1e9, 1)}
    # real-space eigenimages of the selected components (Eq.(IFT_FB) combinations, FP64)
    sel = n_sel.cpu().numpy()
    ks = [k for k in range(plan.k_max + 1) if sel[k] > 0]
    cap = max([int(sel[k]) for k in ks] + [1])
    ebuf = torch.empty((cap, L, L), dtype=torch.complex128, device="cuda")
    plan.eigenimages(evecs, 0, 0, 1, out=ebuf[:1])  # warm-up
    _, e_ms = timed(lambda: [plan.eigenimages(evecs, k, 0, int(sel[k]), out=ebuf[:int(sel[k])]) for k in ks])
    del ebuf
    spca["eigenimages"] = int(sel.sum())
    spca["eigenimages_ms"] = round(e_ms, 3)
    log(f"spca back end: {spca}")

    # adjoint synthesis T a (the differentiation and reconstruction path)
    na = min(n, 16384)
    plan.adjoint(coeffs[:64], batch=pass_images)  # warm-up
    _, adj_ms = timed(lambda: plan.adjoint(coeffs[:na], batch=pass_images))
    adjoint = {"images": na, "ms": round(adj_ms, 3), "images_per_s": round(na / (adj_ms * 1e-3), 1)}
    log(f"adjoint: {adjoint}")

    # estimation of R and c (Sec. VI-C) on a CTF-filtered workload (Eq.(CTFenv), 1 A per pixel,
    # noise at SNR 1/2 over the filtered clean power)
    from paper_1412_0781_amd import workload as wl
    ne = min(n, 20000)
    Hf = wl.ctf_ring_filter(plan)
    clean = wl.synthetic_images(plan, 0, 256, seed=1, snr=1.0, ring_filter=Hf, sigma=0.0)
    sig = float((clean.double().pow(2).mean() / 0.5).sqrt())
    del clean
    imgs_e = wl.synthetic_images(plan, 0, ne, seed=1, snr=1.0, ring_filter=Hf, sigma=sig)
    plan.pixel_moments(imgs_e[:64])  # warm-up

    def estimate_rc():
        s1, s2 = plan.pixel_moments(imgs_e)
        pw = plan.polar_power(imgs_e, pixel_sum=s1, count=ne, batch=pass_images)
        return plan.estimate_support(s1, s2, ne, pw, sig * sig, 0.999)

    (R_est, c_est), est_ms = timed(estimate_rc)
    del imgs_e
    support = {"images": ne, "ms": round(est_ms, 3), "images_per_s": round(ne / (est_ms * 1e-3), 1), "R": R_est,
               "c": round(c_est, 4), "workload": "CTF-filtered synthesis, support R=L/2, SNR 1/2"}
    log(f"support estimate: {support}")
    return {"svd": svd, "spca": spca, "adjoint": adjoint, "support_estimate": support}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--L", type=int, default=None)
    ap.add_argument("--snr", type=float, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--pass-images", type=int, default=2048)
    ap.add_argument("--forms", default=None)
    ap.add_argument("--cpu-sample", type=int, default=None)
    ap.add_argument("--dict-images", type=int, default=None,
                    help="images of the pixel-dictionary accuracy check (0 skips it)")
    ap.add_argument("--dict-pixels", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    wk = WORKLOADS[args.workload]
    for key in ("n", "L", "snr", "forms", "cpu_sample", "dict_images", "dict_pixels"):
        if getattr(args, key) is None:
            setattr(args, key, wk[key])
    kind = wk["kind"]

    import numpy as np
    import torch

    from paper_1412_0781_amd import Plan

    torch.cuda.set_device(0)
    if args.copy_calibration_gib > 0:
        nel = int(args.copy_calibration_gib * (1 << 30)) // 4
        src = torch.empty(nel, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * nel, "copy_bytes_written": 4 * nel}), flush=True)
        return
    L = args.L
    c, R = 0.5, L / 2
    log(f"workload {args.workload} ({kind}): plan L={L} R={R} c={c}")
    t0 = time.perf_counter()
    plan = Plan(L, c, R)
    plan_s = time.perf_counter() - t0
    log(f"plan built in {plan_s:.2f} s: n_xi={plan.n_xi} n_theta={plan.n_theta} k_max={plan.k_max} "
        f"p_half={plan.p_half}")
    plan.workspace(args.pass_images)
    precs = [f.strip() for f in args.forms.split(",") if f.strip()]

    forms, profs = {}, {}
    images = coeffs = st = None
    passes = 1
    steps_done = args.steps
    from paper_1412_0781_amd.workload import noise_sigma
    sigma = noise_sigma(plan, args.snr)
    if kind == "resident":
        log(f"generating {args.n} images on the device")
        t0 = time.perf_counter()
        images, sigma = make_images(plan, args.n, args.seed, args.snr)
        log(f"images ready in {time.perf_counter() - t0:.1f} s (noise sigma {sigma:.4g})")
        coeffs = torch.empty((args.n, plan.p_half, 2), dtype=torch.float32, device=plan.device)
        for prec in precs:
            wall, ev_ms, prof, st = time_form(plan, images, coeffs, prec, args.steps, args.warmup, args.pass_images)
            forms[prec] = {"images_per_s": args.n * args.steps / wall, "ms_per_step": 1e3 * wall / args.steps,
                           "event_ms_per_step": ev_ms / args.steps}
            profs[prec] = prof
        timed_images = args.n * args.steps
        n_step = args.n
    elif kind == "stream":
        for prec in precs:
            ms, nch, prof, st = time_stream(plan, args.n, wk["chunk"], args.seed, args.snr, prec, args.pass_images)
            forms[prec] = {"images_per_s": args.n / (ms * 1e-3), "ms_per_step": ms / nch, "chunks": nch}
            profs[prec] = prof
        steps_done = (args.n + wk["chunk"] - 1) // wk["chunk"]
        timed_images = args.n
        n_step = min(args.n, wk["chunk"])
    else:  # autograd
        wall, ev_ms, prof, sigma = time_autograd(plan, args.n, args.seed, args.snr, args.steps, args.warmup,
                                                 args.pass_images)
        forms["fp32"] = {"images_per_s": args.n * args.steps / wall, "ms_per_step": 1e3 * wall / args.steps,
                         "event_ms_per_step": ev_ms / args.steps}
        profs["fp32"] = prof
        timed_images = args.n * args.steps
        n_step = args.n
        passes = 2  # the backward pass runs the expansion and the synthesis once more
    head = wk["head"] if wk["head"] in forms else next(iter(forms))

    eig_ms = None
    legs = {}
    if st is not None:
        # eigendecomposition of the accumulated covariance (outside images/s)
        torch.cuda.synchronize()
        te = time.perf_counter()
        evals, evecs, _, mean = plan.eig(st)
        torch.cuda.synchronize()
        eig_ms = 1e3 * (time.perf_counter() - te)
        if args.workload == "c3":
            legs = extra_legs(plan, coeffs, evals, evecs, mean, args.n, sigma, args.pass_images)
    del images, coeffs

    stages = _stage_totals(profs[head])
    roofline = kernel_roofline(plan, stages, timed_images * passes, head)
    step = {prec: step_roofline(plan, prec, _stage_totals(profs[prec]), timed_images, forms[prec]["ms_per_step"],
                                n_step, passes)
            for prec in forms}
    log(f"roofline: {roofline}")
    log(f"step roofline: {step}")

    # accuracy on a host-generated sample, and the CPU oracle baseline
    accuracy = None
    cpu = None
    if not args.no_cpu_baseline:
        img_s, coef_ref, po, cpu = cpu_baseline((L, c, R), args.cpu_sample, args.seed, args.snr, kind)
        xs = torch.tensor(img_s, device=plan.device)
        accuracy = {}
        for prec in forms:
            got = plan.expand(xs, precision=prec).cpu().numpy().astype(np.float64)
            gc = got[..., 0] + 1j * got[..., 1]
            accuracy[prec] = {"coeff_rel_l2_workload_sample": float(np.linalg.norm(gc - coef_ref)
                                                                    / np.linalg.norm(coef_ref))}
        log(f"coefficient rel-L2 vs FP64 oracle on the sample: {accuracy}")
        if args.dict_images > 0:
            dict_acc = dictionary_accuracy(plan, po, args.dict_images, args.dict_pixels, list(forms))
            for prec, d in dict_acc.items():
                accuracy[prec].update(d)
            log(f"accuracy vs FP64 oracle (pixel-dictionary images): {accuracy}")

    f = forms[head]
    what = {"resident": "FB expansion + covariance",
            "stream": f"FB expansion + covariance, streamed in chunks of {wk.get('chunk')}",
            "autograd": "FB expansion, shrinkage, synthesis, forward + backward"}[kind]
    metric = METRIC if args.workload == "c3" else \
        f"images/s ({what}) at L={L}, " + ("FP32" if kind == "autograd" else "BF16x3 vs FP32")
    out = {
        "metric": metric,
        "value": round(f["images_per_s"], 1),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": steps_done,
        "warmup": args.warmup,
        "ms_per_step": round(f["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (autograd path)" if kind == "autograd" else f"{head} matrix-core contractions, f32 NUFFT",
        "data": "synthetic",
        "config": {"workload": f"{what}, n={args.n} images L={L} R={R:g} c={c} "
                               f"SNR=1/{round(1 / args.snr)} (synthetic, device-generated, seed {args.seed})",
                   "name": args.workload, "n": args.n, "L": L, "R": R, "c": c, "precision": head,
                   "pass_images": args.pass_images},
        "forms": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in forms.items()},
        "bf16x3_over_fp32": round(forms["bf16x3"]["images_per_s"] / forms["fp32"]["images_per_s"], 3)
        if "bf16x3" in forms and "fp32" in forms else None,
        "accuracy_rel_l2": accuracy,
        "stages": {k: {kk: round(vv, 4) if isinstance(vv, float) else vv for kk, vv in v.items()}
                   for k, v in stages.items()},
        "eig_ms": round(eig_ms, 2) if eig_ms is not None else None,
        **legs,
        "plan_s": round(plan_s, 2),
        "roofline": roofline,
        "step_roofline": step,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
