#!/usr/bin/env python3
"""Throughput of dense membrane-probability inference on one MI355X.

Headline: the plain net B in FP32 over a 32 x 1024 x 1024 uint8 EM-like volume
(seeded synthetic stand-in for the paper's EM stacks), one step = one dense pass
of the whole path (uint8 ingest, conv1 + ReLU, 2x2/s1 max filter, conv2 + ReLU,
max filter, conv3 + ReLU, 1x1 head + sigmoid) with input and output resident in
HBM. Printed as one JSON line; also reported:

* roofline of the dominant kernel (conv2, 72% of the FLOPs) from HIP events
  recorded on its launch stream over the timed region;
* the FP64 CPU reference timed on a bounded sample on the host cores;
* the other forms (BF16 / FP8 precision, batched tiles, student, and the
  paper's own FastMemb net in FP32 on the same volume) unless --forms none.

Only one GPU is used; --gpus N with N > 1 is refused.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "membrane-prob voxels/sec at 1 MI355X and % MFMA peak, plain FP32 vs BF16/FP8/student"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
HBM_GBS = 8000.0
# algorithmic work of net B per output voxel: 2 x (1200 + 57600 + 20736 + 48) MAC
NET_B_FLOP_PER_VOXEL = 159168
CONV2_FLOP_PER_POS = 2 * 25 * 48 * 48  # per conv2 output position
CONV1_FLOP_PER_POS = 2 * 25 * 48  # per conv1 output position
CONV3_FLOP_PER_POS = 2 * 9 * 48 * 48 + 2 * 48  # per conv3 output position, head included
STUDENT_FLOP_PER_VOXEL = 2 * (200 + 576 + 8)
# FastMemb (4x4 convs 1->64, 32->64, 32->64 with max-out to 32, 32->2) per output voxel
FASTMEMB_FLOP_PER_VOXEL = 2 * 16 * (64 + 32 * 64 + 32 * 64 + 32 * 2)
FASTMEMB_BODY_FLOP_PER_POS = 2 * 16 * 32 * 64  # one 32 -> 64 4x4 conv output position
# FastMemb_ss per 6 nm output voxel: the 1 -> 64 conv only where the subsample keeps pixels, three 32 -> 64 convs
FASTMEMB_SS_FLOP_PER_VOXEL = 2 * 16 * (64 + 3 * 32 * 64 + 32 * 2)
# MaskExtend per output voxel: five 4x4 convs (12->64, 32->80, 40->96, 48->112, 56->128), 1x1 64->3
MASKEXTEND_FLOP_PER_VOXEL = 2 * 16 * (12 * 64 + 32 * 80 + 40 * 96 + 48 * 112 + 56 * 128) + 2 * 64 * 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    """sha1 of the conv kernels' source and of the build script (its per-file
    compiler flags change the code of the same source)."""
    h = hashlib.sha1()
    for f in ("csrc/conv_kernels.hip", "build_lib.py"):
        with open(os.path.join(ROOT, "paper_1612_02120_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_from_profiles(name):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        if d.get("kernel_source_sha") != kernel_source_sha():
            return None
        return d.get("hbm_bytes_per_launch")
    except Exception:
        return None


def time_volume(emcnn, torch, h, vol_dev, steps, warmup, stream):
    Ho, Wo = h.out_dims(vol_dev.shape[1], vol_dev.shape[2])
    out = torch.empty((vol_dev.shape[0], Ho, Wo), dtype=torch.float32, device=vol_dev.device)
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            emcnn.cnn_infer(h, vol_dev, out=out, stream=stream)
        torch.cuda.synchronize()
        emcnn.cnn_profile_read(h)  # clear
        emcnn.cnn_profile(h, True)
        t0 = time.perf_counter()
        for _ in range(steps):
            emcnn.cnn_infer(h, vol_dev, out=out, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        emcnn.cnn_profile(h, False)
    ms, n = emcnn.cnn_profile_read(h)
    # per pass: a volume larger than the handle's slab budget runs each layer
    # once per slab, and a pass is all of them
    per_layer = [m / steps for m in ms]
    time_volume.launches_per_pass = [c / steps for c in n]
    return (t1 - t0) * 1e3 / steps, per_layer, out


def _oracle_rate(vol, net, params, min_seconds, threads, native):
    """Output voxels/s of the FP64 oracle over whole slices (or the given
    window) of `vol`, one slice after another until min_seconds have run."""
    import oracle
    R = oracle.radius(net)
    nvox, n, t0 = 0, 0, time.perf_counter()
    while n < vol.shape[0]:
        oracle.forward(np.ascontiguousarray(vol[n:n + 1]), net, params, threads=threads, native=native)
        nvox += (vol.shape[1] - R) * (vol.shape[2] - R)
        n += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    return nvox / (time.perf_counter() - t0), n, nvox, time.perf_counter() - t0


def cpu_baseline(vol, net, params, out_vox_unit="voxels/s"):
    """The FP64 CPU oracle on the host cores, on a bounded sample of the
    benchmark volume: its -O3 -march=native timing build (compiled for this
    host; bitwise the same results as the test build) on all threads over whole
    1024^2 slices, on one thread over a 140-row window of slice 0, and the -O2
    test build on all threads for comparison."""
    import oracle
    from oracle import build as oracle_build
    threads = oracle.num_threads()
    native_ok = True
    try:
        oracle.native_lib()
    except Exception as e:  # no compiler on the host: time the test build only
        log("oracle timing build unavailable (%s); timing the -O2 test build" % e)
        native_ok = False
    v_all, n_all, vox_all, dt_all = _oracle_rate(vol, net, params, 8.0, threads, native_ok)
    win = np.ascontiguousarray(vol[:1, :140, :])
    v_one, _, vox_one, dt_one = _oracle_rate(win, net, params, 0.0, 1, native_ok)
    v_o2, n_o2, _, dt_o2 = _oracle_rate(vol, net, params, 4.0, threads, False)
    build = ("-O3 -march=native -ffp-contract=off (timing build)" if native_ok else
             "-O2 -ffp-contract=off (test build)")
    return {"value": v_all, "unit": out_vox_unit, "cores": threads, "kind": "oracle",
            "cpu_model": oracle_build.cpu_model(), "host_nproc": os.cpu_count(),
            "build": build,
            "value_1_thread": v_one,
            "value_o2_test_build": v_o2,
            "sample": "%d whole slice(s) of the benchmark volume (%d x %d) -> %d output voxels in %.1f s on %d "
                      "threads; 1 thread: slice 0 rows 0..139 -> %d output voxels in %.1f s; -O2 test build: "
                      "%d slice(s) in %.1f s; FP64 direct convolution"
                      % (n_all, vol.shape[1], vol.shape[2], vox_all, dt_all, threads, vox_one, dt_one, n_o2, dt_o2)}


def student_form(emcnn, torch, em_volume, p, NET_B, dev, stream, args, big):
    """Distil the student (64 volumes of 16 x 512 x 512, Adam lr 1e-3, batch 16 x
    128^2; 20k steps, 4k with --quick) from the FP32 net's maps, then on the
    evaluation volume `big` (the precision volume, 128 x 2048^2 by default) time
    the student, the plain net in FP32 and BF16, and student + fallback over a
    grid of fallback tile sizes and thresholds tau, with agreement and fallback
    rate at each point."""
    from paper_1612_02120_amd import distill
    from synth.nets import NET_S, he_normal_params
    steps = 4000 if args.quick else 20000
    t0 = time.perf_counter()
    vols = [torch.from_numpy(em_volume(5000 + i, 16, 512, 512)).to(dev) for i in range(64)]
    teacher = emcnn.cnn_create(p, NET_B, "fp32")
    maps = distill.teacher_maps(teacher, vols)
    s = emcnn.student_create(he_normal_params(NET_S, 300), "bf16")
    losses, _ = distill.train(s, vols, maps, teacher.R, steps, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del vols, maps
    Zs = big.shape[0]
    tmap = emcnn.cnn_infer(teacher, big)
    b16 = emcnn.cnn_create(p, NET_B, "bf16")
    nv = Zs * (big.shape[1] - teacher.R) * (big.shape[2] - teacher.R)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / reps

    t_s = timed(lambda: emcnn.student_infer(s, big, stream=stream))
    t32 = timed(lambda: emcnn.cnn_infer(teacher, big, stream=stream))
    t16 = timed(lambda: emcnn.cnn_infer(b16, big, stream=stream))
    v32, v16 = nv / t32, nv / t16
    raw, _, _ = distill.evaluate(s, teacher, big, tmap, tau=1.0, tile=512, n_samples=1, seed=3)
    res = {"workload": "student conv5x5 1->8, conv3x3 8->8, 1x1 sigmoid, BF16; distilled %d steps "
                       "(64 x 16 x 512^2, batch 16 x 128^2, lr 1e-3) from FP32 net B; eval %d x %d x %d (seed 3)"
                       % (steps, Zs, big.shape[1], big.shape[2]),
           "train_s": t_train, "final_loss": float(losses[-200:].mean().item()),
           "student_voxels_per_s": nv / t_s,
           "student_tflops": nv * STUDENT_FLOP_PER_VOXEL / t_s / 1e12,
           "student_mfma_frac": nv * STUDENT_FLOP_PER_VOXEL / t_s / 1e12 / PEAK_TFLOPS["bf16"],
           "raw_agreement": raw["raw_agreement"],
           "net_b_fp32_voxels_per_s": v32, "net_b_bf16_voxels_per_s": v16,
           "bf16_teacher_agreement_with_fp32": distill.agreement(emcnn.cnn_infer(b16, big), tmap)}
    grid = []
    for tile in (64, 128, 256, 512):
        ns = max(1, tile // 64)  # sampled windows grow with the tile
        for tau in (0.0, 0.01, 0.05, 0.1, 0.25):
            r, out, st = distill.evaluate(s, teacher, big, tmap, tau=tau, tile=tile, n_samples=ns, seed=3)
            del out
            t_f = timed(lambda: emcnn.student_infer_with_fallback(s, teacher, big, tau=tau, tile=tile,
                                                                  n_samples=ns, seed=3, stream=stream), reps=1)
            pt = {"tile": tile, "n_samples": ns, "tau": tau, "fallback_rate": r["fallback_rate"],
                  "agreement": r["agreement"], "voxels_per_s": nv / t_f}
            grid.append(pt)
            log("student fallback", json.dumps(pt))
    res["fallback_grid"] = grid
    ok = [g for g in grid if g["agreement"] >= 0.99]
    best = max(ok, key=lambda g: g["voxels_per_s"]) if ok else None
    res["target_0.99"] = {
        "met_by": best, "beats_fp32_net_b": bool(best and best["voxels_per_s"] > v32),
        "beats_bf16_net_b": bool(best and best["voxels_per_s"] > v16),
        "best_point_any_agreement": max(grid, key=lambda g: g["agreement"] - 1e-12 * g["voxels_per_s"])}
    return res


def fastmemb_ss_form(emcnn, torch, em_volume, calibrated_params, dev, stream, args, forms):
    """FastMemb_ss (Section 2.2, "A subsampling CNN for 3 nm data"; the reading:
    FastMemb plus one more {pool, conv} pair with its first stride-2 pool
    replaced by a 2x subsample) on a 32 x 2048 x 2048 stack taken as 3 nm
    sections, giving a 32 x 971 x 971 map at 6 nm: the same output size as
    FastMemb on 32 x 1024^2 (6 nm sections). Reports the closed-form cost
    ratio to FastMemb_6nm beside the paper's figure, and the measured one."""
    from synth.nets import NET_FMSS, he_normal_params
    Z = 32
    vol = torch.from_numpy(em_volume(5, Z, 2048, 2048)).to(dev)
    p = he_normal_params(NET_FMSS, 410)
    out = {}
    for prec in ("fp32", "bf16"):
        h = emcnn.cnn_create(p, NET_FMSS, prec)
        ms, pl, o = time_volume(emcnn, torch, h, vol, max(3, args.steps // 2), 2, stream)
        nv = o.numel()
        out[prec] = {"voxels_per_s": nv / (ms * 1e-3), "ms_per_pass": ms, "output": list(o.shape),
                     "path_tflops": nv * FASTMEMB_SS_FLOP_PER_VOXEL / (ms * 1e-3) / 1e12,
                     "path_mfma_frac": nv * FASTMEMB_SS_FLOP_PER_VOXEL / (ms * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                     "layer_ms": pl[:5], "tiles": emcnn.cnn_describe(h)}
        fm = forms.get("fastmemb" if prec == "fp32" else "fastmemb_bf16")
        if fm:
            out[prec]["time_ratio_vs_fastmemb_6nm"] = ms / fm["ms_per_pass"] * (32 * 972 ** 2) / nv
        del o, h
    res = {"workload": "FastMemb_ss (conv4x4 1->64 max-out, 2x subsample, conv4x4 32->64 max-out, 3 x {2x2/s2 "
                       "pool, conv4x4}, two-class softmax; FoV 108 at 3 nm) on %d x 2048 x 2048 (seed 5) -> "
                       "%d x 971 x 971 at 6 nm" % (Z, Z),
           "flop_ratio_vs_fastmemb_6nm": FASTMEMB_SS_FLOP_PER_VOXEL / FASTMEMB_FLOP_PER_VOXEL,
           "paper_flop_ratio": 1.17, **out}
    log("fastmemb_ss", json.dumps(res))
    return res


def maskextend_form(emcnn, torch, dev, stream, args):
    """MaskExtend (Section 3; the reading in the design notes) in FP32 on
    8 x 1024 x 1024 sections of twelve synthetic input maps (EM, object masks,
    membrane maps; synth.maskextend_maps) -> 8 x 916 x 916 object probabilities."""
    from synth import maskextend_maps
    from synth.nets import NET_ME, he_normal_params
    Z = 4 if args.quick else 8
    t0 = time.perf_counter()
    maps = torch.from_numpy(maskextend_maps(6, Z, 1024, 1024)).to(dev)
    log("generated MaskExtend maps %s in %.1fs" % (tuple(maps.shape), time.perf_counter() - t0))
    h = emcnn.cnn_create(he_normal_params(NET_ME, 500), NET_ME, "fp32")
    out = emcnn.cnn_infer_maps(h, maps)
    torch.cuda.synchronize()
    reps = max(3, args.steps // 2)
    with torch.cuda.stream(stream):
        emcnn.cnn_infer_maps(h, maps, out=out, stream=stream)
        torch.cuda.synchronize()
        emcnn.cnn_profile_read(h)
        emcnn.cnn_profile(h, True)
        t0 = time.perf_counter()
        for _ in range(reps):
            emcnn.cnn_infer_maps(h, maps, out=out, stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        emcnn.cnn_profile(h, False)
    ms, n = emcnn.cnn_profile_read(h)
    nv = out.numel()
    res = {"workload": "MaskExtend FP32 (12 input maps; 4x4 max-out convs to 32/40/48/56/64 features with 2x2/s2 "
                       "pools; 1x1 three-class softmax; FoV 109) on %d x 1024 x 1024 x 12 -> %d x 916 x 916"
                       % (Z, Z),
           "voxels_per_s": nv / dt, "ms_per_pass": dt * 1e3,
           "path_tflops": nv * MASKEXTEND_FLOP_PER_VOXEL / dt / 1e12,
           "path_mfma_frac": nv * MASKEXTEND_FLOP_PER_VOXEL / dt / 1e12 / PEAK_TFLOPS["fp32"],
           "layer_ms": [m / reps for m in ms[:6]], "tiles": emcnn.cnn_describe(h)}
    log("maskextend", json.dumps(res))
    del maps, out, h
    return res


def watershed_form(emcnn, torch, pmap, stream, reps=5):
    """The 3-D watershed (Section 2.1, over-segmentation) on the headline
    membrane map (32 x 1012 x 1012 FP32), seeds below its 25 % quantile.
    Algorithmic traffic: 4 B read + 4 B written per voxel."""
    t = float(torch.quantile(pmap[0].flatten()[::97].float(), 0.25).item())
    lab = torch.empty(pmap.shape, dtype=torch.int32, device=pmap.device)
    work = torch.empty(pmap.numel() + 1, dtype=torch.int32, device=pmap.device)
    with torch.cuda.stream(stream):
        emcnn.watershed_3d(pmap, t, labels=lab, work=work, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            emcnn.watershed_3d(pmap, t, labels=lab, work=work, stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
    n = pmap.numel()
    nb = int(torch.unique(lab).numel())
    res = {"workload": "3-D watershed (steepest descent, seeded minima, 6-neighbours) of the net B FP32 map "
                       "%s, seeds p < %.4f" % (tuple(pmap.shape), t),
           "voxels_per_s": n / dt, "ms_per_pass": dt * 1e3, "basins": nb,
           "roofline": {"bound": "hbm", "achieved": n * 8 / dt / 1e9, "peak": HBM_GBS, "unit": "GB/s",
                        "frac": n * 8 / dt / 1e9 / HBM_GBS, "algorithmic_bytes_per_voxel": 8}}
    log("watershed", json.dumps(res))
    return res


def mfma_ceiling(emcnn, torch, dev):
    """Measured MFMA throughput of each precision's instruction on random
    operands (register operands, 8 accumulators per wave, 16 waves per CU),
    with the shader clock the waves ran at."""
    rng = np.random.default_rng(7)
    out = {}
    for prec in ("fp32", "bf16", "fp8"):
        ops = rng.integers(0, 256, size=(256 * 2 * 64 * 32,)).astype(np.uint8)
        if prec == "fp8":
            ops[ops == 0x7F] = 0x7E  # no NaN codes
            ops[ops == 0xFF] = 0xFE
        elif prec == "bf16":
            ops[1::2] &= 0xBF  # finite bf16 values (exponent below the top half)
        else:
            ops[3::4] &= 0xBF
        tf, mhz = emcnn.cnn_mfma_bench(prec, torch.from_numpy(ops).to(dev), blocks=4096, iters=2048)
        out[prec] = {"tflops": tf, "frac_of_vendor_peak": tf / PEAK_TFLOPS[prec], "shader_mhz": mhz,
                     "vendor_peak_tflops": PEAK_TFLOPS[prec]}
        log("mfma ceiling", prec, json.dumps(out[prec]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default="all",
                    help="all | none | comma list of mfma,watershed,bf16,fp8,batch,student,fastmemb,"
                         "fastmemb_bf16,fastmemb_ss,maskextend")
    ap.add_argument("--quick", action="store_true",
                    help="smaller secondary forms: precision / student volume 8 x 2048^2, 4k training steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate tile shapes first for the FP32 / BF16 / FP8 volumes "
                         "(the defaults are the measured best); the batched form always autotunes")
    ap.add_argument("--no-batch-autotune", action="store_true", help="batched form with the default tiles")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (read, then updated)")
    ap.add_argument("--no-headline", action="store_true", help="skip the FP32 headline (profiling runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one 1 GiB device-to-device copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1612_02120_amd as emcnn
    from synth import em_volume
    from synth.nets import NET_B, calibrated_params, fp8_act_scales

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    if args.copy_calib:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    Z, H, W = 32, 1024, 1024
    if args.no_headline:
        Z = 1
    t0 = time.perf_counter()
    vol = em_volume(2, Z, H, W)
    log("generated %s volume in %.1fs" % ((Z, H, W), time.perf_counter() - t0))
    vol_dev = torch.from_numpy(vol).to(dev)
    p = calibrated_params("B")
    h = emcnn.cnn_create(p, NET_B, "fp32")
    if args.autotune:
        emcnn.cnn_autotune(h, H, W, args.tune_cache, stream)
    R = h.R
    Ho, Wo = H - R, W - R
    nvox = Z * Ho * Wo
    ms, per_layer, out = time_volume(emcnn, torch, h, vol_dev, 1 if args.no_headline else args.steps,
                                     0 if args.no_headline else args.warmup, stream)
    value = nvox / (ms * 1e-3)
    if time_volume.launches_per_pass[1] != 1:
        raise SystemExit("headline volume must run as one slab (one conv2 launch per pass)")
    conv2_ms = per_layer[1]
    conv2_units = Z * (H - 9) * (W - 9)
    conv2_flop = conv2_units * CONV2_FLOP_PER_POS
    achieved = conv2_flop / (conv2_ms * 1e-3) / 1e12 if conv2_ms > 0 else None
    path_tflops = nvox * NET_B_FLOP_PER_VOXEL / (ms * 1e-3) / 1e12
    log("fp32: %.3f ms/step, %.3e vox/s, layers ms %s, tiles %s" %
        (ms, value, ["%.3f" % x for x in per_layer[:3]], emcnn.cnn_describe(h)))
    res = {
        "metric": METRIC, "value": value, "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plain net B FP32, dense over 32 x 1024 x 1024 uint8 EM-like volume "
                               "(seed 2) -> 32 x 1012 x 1012 probabilities",
                   "net": "conv5x5 1->48, pool2x2/s1, conv5x5 48->48, pool2x2/s1, conv3x3 48->48, "
                          "conv1x1 48->1 sigmoid",
                   "precision": "fp32", "output_voxels": nvox, "tiles": emcnn.cnn_describe(h)},
        "path_mfma_frac": path_tflops / PEAK_TFLOPS["fp32"],
        "path_tflops": path_tflops,
        "layer_ms": per_layer[:3],
        "roofline": {"bound": "mfma", "kernel": "conv2 (conv_mfma FP32 48->48 5x5, pool fused)",
                     "achieved": achieved, "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                     "frac": (achieved / PEAK_TFLOPS["fp32"]) if achieved else None,
                     "flop_per_launch": conv2_flop, "avg_launch_ms": conv2_ms,
                     "traffic": traffic_from_profiles("conv2_fp32_plain_traffic.json")},
    }
    forms = {}
    if args.forms == "all" or "watershed" in args.forms.split(","):
        forms["watershed"] = watershed_form(emcnn, torch, out, stream)
    del out
    want = set() if args.forms == "none" else (
        {"mfma", "bf16", "fp8", "batch", "student", "fastmemb", "fastmemb_bf16", "fastmemb_ss", "maskextend"}
        if args.forms == "all"
        else set(args.forms.split(",")))
    if "mfma" in want:
        forms["mfma_ceiling"] = mfma_ceiling(emcnn, torch, dev)
    for fm_prec in ("fp32", "bf16"):
        key = "fastmemb" if fm_prec == "fp32" else "fastmemb_bf16"
        if key not in want or args.no_headline:
            continue
        # the paper's own net (Section 2.2) on the headline volume: dense form of
        # its stride-2 pools (max filters, convs spaced 2, 4, 8 over phase sub-lattices)
        from synth.nets import NET_FM
        hf = emcnn.cnn_create(calibrated_params("FM"), NET_FM, fm_prec)
        msf, plf, outf = time_volume(emcnn, torch, hf, vol_dev, max(3, args.steps // 2), 2, stream)
        nvf = Z * (H - hf.R) * (W - hf.R)
        body_flop = [Z * (H - 3 - 7) ** 2 * FASTMEMB_BODY_FLOP_PER_POS,
                     Z * (H - 3 - 7 - 14) ** 2 * FASTMEMB_BODY_FLOP_PER_POS]
        body_tf = [f / (t * 1e-3) / 1e12 for f, t in zip(body_flop, plf[1:3])]
        forms[key] = {
            "workload": "FastMemb %s (conv4x4 1->64 max-out, 3 x {2x2/s2 pool, conv4x4}, two-class softmax; "
                        "FoV 53), %d x %d x %d (seed 2) -> %d x %d x %d"
                        % (fm_prec.upper(), Z, H, W, Z, H - hf.R, W - hf.R),
            "voxels_per_s": nvf / (msf * 1e-3), "ms_per_pass": msf,
            "path_mfma_frac": nvf * FASTMEMB_FLOP_PER_VOXEL / (msf * 1e-3) / 1e12 / PEAK_TFLOPS[fm_prec],
            "body_conv_tflops": body_tf, "body_conv_frac": [t / PEAK_TFLOPS[fm_prec] for t in body_tf],
            "layer_ms": plf[:4], "tiles": emcnn.cnn_describe(hf)}
        log(key, json.dumps(forms[key]))
        del outf, hf
    if "maskextend" in want:
        forms["maskextend"] = maskextend_form(emcnn, torch, dev, stream, args)
    if "fastmemb_ss" in want and not args.no_headline:
        forms["fastmemb_ss"] = fastmemb_ss_form(emcnn, torch, em_volume, calibrated_params, dev, stream, args,
                                                forms)
    volp_dev = None
    if want & {"bf16", "fp8", "student"}:
        Zp = 8 if args.quick else 128
        t0 = time.perf_counter()
        volp = em_volume(3, Zp, 2048, 2048)
        log("generated precision volume %s in %.1fs" % ((Zp, 2048, 2048), time.perf_counter() - t0))
        volp_dev = torch.from_numpy(volp).to(dev)
        del volp
        nv = Zp * (2048 - R) ** 2
    if want & {"bf16", "fp8"}:
        for prec in ("bf16", "fp8"):
            if prec not in want:
                continue
            hp = emcnn.cnn_create(p, NET_B, prec,
                                  act_scales=fp8_act_scales("B") if prec == "fp8" else None)
            if args.autotune:
                emcnn.cnn_autotune(hp, 2048, 2048, args.tune_cache, stream)
            msp, pl, outp = time_volume(emcnn, torch, hp, volp_dev, max(3, args.steps // 2), 2, stream)
            c2u = Zp * (2048 - 9) ** 2
            flop2 = c2u * CONV2_FLOP_PER_POS
            fused = pl[0] == 0.0  # layer 0 computed inside the conv2 kernel
            if fused:
                flop2 += Zp * (2048 - 4) ** 2 * CONV1_FLOP_PER_POS
            ach = flop2 / (pl[1] * 1e-3) / 1e12
            ach3 = Zp * (2048 - 12) ** 2 * CONV3_FLOP_PER_POS / (pl[2] * 1e-3) / 1e12
            ceil = forms.get("mfma_ceiling", {}).get(prec, {}).get("tflops")
            forms[prec] = {"workload": "net B %s, %d x 2048 x 2048 (seed 3)" % (prec, Zp),
                           "voxels_per_s": nv / (msp * 1e-3), "ms_per_pass": msp,
                           "path_mfma_frac": nv * NET_B_FLOP_PER_VOXEL / (msp * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                           "conv2_tflops": ach, "conv2_frac": ach / PEAK_TFLOPS[prec],
                           "conv3_tflops": ach3, "conv3_frac": ach3 / PEAK_TFLOPS[prec],
                           "conv2_frac_of_measured_ceiling": ach / ceil if ceil else None,
                           "conv3_frac_of_measured_ceiling": ach3 / ceil if ceil else None,
                           "conv2_kernel_includes_conv1": fused, "layer_ms": pl[:3],
                           "slabs_per_pass": time_volume.launches_per_pass[2],
                           "tiles": emcnn.cnn_describe(hp)}
            log(prec, json.dumps(forms[prec]))
            del outp, hp
    if "batch" in want:
        from synth import batch_tiles
        tl = batch_tiles()
        rng = np.random.default_rng(44)
        pool = em_volume(4, 8, 1040, 1040)
        hb = emcnn.cnn_create(p, NET_B, "bf16")
        t_tune = 0.0
        tiles, nv = [], 0
        for t in tl:
            y = int(rng.integers(0, 1040 - t["h"] + 1))
            x = int(rng.integers(0, 1040 - t["w"] + 1))
            inp = torch.from_numpy(np.ascontiguousarray(pool[:t["z"], y:y + t["h"], x:x + t["w"]])).to(dev)
            L = t["h"] - 2 * t["halo"]
            out = torch.empty((t["z"], L, L), dtype=torch.float32, device=dev)
            tiles.append((inp, t["halo"], out))
            nv += t["z"] * L * L
        if not args.no_batch_autotune:  # tile shapes per tile class, tuned on these tiles
            t0 = time.perf_counter()
            emcnn.cnn_autotune_batch(hb, tiles, stream)
            t_tune = time.perf_counter() - t0
        with torch.cuda.stream(stream):
            for _ in range(2):
                emcnn.cnn_infer_batch(hb, tiles, stream=stream)
            torch.cuda.synchronize()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                emcnn.cnn_infer_batch(hb, tiles, stream=stream)
            torch.cuda.synchronize()
            msb = (time.perf_counter() - t0) * 1e3 / reps
            # per-tile loop: cnn_infer on each tile's input cropped to a halo of R/2
            # (copied contiguous before timing), one direct launch per layer
            e = 8 - R // 2
            cropped = [(inp[:, e:inp.shape[1] - e, e:inp.shape[2] - e].contiguous(), out) for (inp, _, out) in tiles]
            for (cin_, out) in cropped[:4]:
                emcnn.cnn_infer(hb, cin_, out=out, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for (cin_, out) in cropped:
                emcnn.cnn_infer(hb, cin_, out=out, stream=stream)
            torch.cuda.synchronize()
            msl = (time.perf_counter() - t0) * 1e3
            del cropped
        forms["batch"] = {"workload": "512 tiles, side logU[64,1024], 1-8 slices, halo 8, BF16 net B",
                          "output_voxels": nv, "voxels_per_s_graph": nv / (msb * 1e-3),
                          "ms_graph": msb, "voxels_per_s_per_tile_loop": nv / (msl * 1e-3),
                          "ms_per_tile_loop": msl,
                          "per_tile_loop": "cnn_infer per tile (input cropped to a halo of R/2), 3 direct "
                                           "launches per tile, no host waits",
                          "path_mfma_frac": nv * NET_B_FLOP_PER_VOXEL / (msb * 1e-3) / 1e12 / PEAK_TFLOPS["bf16"],
                          "autotuned": "per tile class" if not args.no_batch_autotune else False, "autotune_s": t_tune,
                          "tiles": emcnn.cnn_describe(hb)}
        log("batch", json.dumps(forms["batch"]))
        del tiles, hb
    if "student" in want:
        forms["student"] = student_form(emcnn, torch, em_volume, p, NET_B, dev, stream, args, volp_dev)
        log("student", json.dumps(forms["student"]))
    if forms:
        res["forms"] = forms
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(vol, NET_B, p)
        log("cpu baseline", json.dumps(res["cpu_baseline"]))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
