#!/usr/bin/env python3
"""Benchmark of the VoGE rendering hot path on one MI355X.

One step = forward + backward of one 512x512 render of the 10,000-kernel
torus (16 channels, K = 20, eta = 0.01) through the C ABI, with every input
already resident in device memory.  Prints ONE JSON line on stdout:

  value      Mrays/s of forward + backward (rays = pixels per step / step time)
  latency    p50 / p99 of the per-step time (each step is one request)
  roofline   the dominant kernel's algorithmic FLOP rate against the FP32
             vector peak, its average duration measured live with HIP events
  cpu_baseline  the FP64 oracle, forward + backward on a fixed random sample of
             the same image's rays, timed on this host's cores

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--cpu-sample RAYS]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3    # MI355X FP32 vector peak (256 CUs, 2.4 GHz)
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest() -> str:
    h = hashlib.sha256()
    for f in ("trace.hip", "voge_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2205_15401_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, digest: str):
    """HBM bytes per launch from a committed counter summary, if it was taken
    on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_d = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_d or not m_b or m_d.group(1) != digest:
        return None
    return float(m_b.group(1))


def cpu_baseline(job, n_rays: int, seed: int = 7):
    """FP64 oracle, forward + backward, on a fixed random sample of the rays."""
    import numpy as np
    from oracle import oracle as O

    cam = job.camera
    H, W, C = cam.height, cam.width, job.scene.channels
    rng = np.random.default_rng(seed)
    n = min(int(n_rays), H * W)
    pix = np.sort(rng.choice(H * W, n, replace=False))
    G = job.grad_image.reshape(-1, C)[pix]
    threads = len(os.sched_getaffinity(0))
    env_t = os.environ.get("OMP_NUM_THREADS")
    if env_t and env_t.isdigit():
        threads = min(threads, int(env_t))
    t0 = time.perf_counter()
    O.forward(job.scene.means, job.scene.covs, job.scene.attrs, cam.as_vector(), H, W, job.K, job.eta,
              pixels=pix, threads=threads)
    O.backward(job.scene.means, job.scene.covs, job.scene.attrs, cam.as_vector(), H, W, job.K, G, job.eta,
               pixels=pix, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": n / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} random rays of the {H}x{W} image (seed {seed}), forward + backward, "
                      f"brute force over all {job.scene.n} kernels, FP64, {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=131072, help="rays for the oracle baseline (0 = skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="after timing, copy this many bytes device-to-device once (a plain copy kernel of "
                         "known size that scales the HBM byte counters of a profile)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        log("bench.py measures one GPU: this build renders on a single MI355X; "
            "multi-GPU runs are not part of it (see DESIGN.md for how the path would shard).")
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2205_15401_amd import _native as nat
    from paper_2205_15401_amd import render as R
    from paper_2205_15401_amd import scenes as S

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    dev = torch.device("cuda:0")
    job = S.config_torus()
    sc, cam = job.scene, job.camera
    N, C, H, W, K = sc.n, sc.channels, cam.height, cam.width, job.K
    log(f"[bench] workload {job.name}: N={N} C={C} {H}x{W} K={K}")

    means = torch.from_numpy(sc.means).to(dev)
    covs = torch.from_numpy(sc.covs).to(dev)
    attrs = torch.from_numpy(sc.attrs).to(dev)
    grad = torch.from_numpy(job.grad_image).to(dev)
    cs = R.camera_struct(cam)
    par = R.params_struct(K, job.eta)
    ws_bytes = nat.voge_workspace_size(N, C, cs, par, True)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    image = torch.empty((H, W, C), dtype=torch.float32, device=dev)
    gm = torch.empty((N, 3), dtype=torch.float32, device=dev)
    gc = torch.empty((N, 6), dtype=torch.float32, device=dev)
    ga = torch.empty((N, C), dtype=torch.float32, device=dev)
    gk = torch.empty(15, dtype=torch.float32, device=dev)
    ctx = R.context(dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    p = lambda t: t.data_ptr()  # noqa: E731

    def step():
        nat.voge_render_forward(ctx, p(means), p(covs), p(attrs), N, C, cs, par, p(image), None, None, p(ws),
                                ws_bytes, stream)
        nat.voge_render_backward(ctx, p(means), p(covs), p(attrs), N, C, cs, par, p(grad), p(gm), p(gc), p(ga),
                                 p(gk), nat.VOGE_REUSE_PREP, p(ws), ws_bytes, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = nat.voge_status(p(ws), stream)
    if st != 0:
        log(f"[bench] device status {st}")

    nat.voge_profile_enable(ctx, True)
    nat.voge_profile_read(ctx, reset=True)
    events = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    events[0].record()
    for i in range(args.steps):
        step()
        events[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = nat.voge_profile_read(ctx, reset=True)
    nat.voge_profile_enable(ctx, False)
    per_step = np.array([events[i].elapsed_time(events[i + 1]) for i in range(args.steps)])
    if args.calibrate_copy > 0:
        n4 = args.calibrate_copy // 4
        src = torch.ones(n4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {n4 * 4} bytes done")
        del src, dst
    total_ms = events[0].elapsed_time(events[-1])
    ms_per_step = total_ms / args.steps
    rays = H * W
    value = rays / (ms_per_step / 1e3) / 1e6
    log(f"[bench] {args.steps} steps in {total_ms:.2f} ms (wall {wall * 1e3:.1f} ms): {ms_per_step:.4f} ms/step, "
        f"{value:.1f} Mrays/s")
    for name, (tot, cnt) in sorted(phases.items()):
        log(f"[bench]   phase {name:9s} {tot / max(cnt, 1) * 1e3:9.2f} us avg over {cnt}")

    # roofline of the dominant kernel (FLOP counts from the oracle's op counter)
    opc_path = os.path.join(ROOT, "oracle", f"opcount_{job.name}.json")
    roofline = None
    if os.path.exists(opc_path):
        opc = json.load(open(opc_path))
        flops = {"select": opc["flop_select"], "blend": opc["flop_blend"], "bwd": opc["flop_bwd_pixel"],
                 "bwd_reduce": opc["flop_bwd_chain"]}
        kb = R_kb(K)
        kname = {"select": f"k_select<{kb}>", "blend": f"k_blend<{kb}>", "bwd": f"k_bwd_pix<{kb}>",
                 "bwd_reduce": f"k_bwd_red<{kb}>"}
        avg = {k: phases[k][0] / phases[k][1] for k in flops if k in phases and phases[k][1] > 0}
        dom = max(avg, key=avg.get)
        achieved = flops[dom] / (avg[dom] / 1e3) / 1e12
        traffic = load_traffic(kname[dom].split("<")[0], job.name, source_digest())
        roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / PEAK_FP32_TFLOPS, 6), "traffic": traffic,
                    "kernel": kname[dom], "avg_us": round(avg[dom] * 1e3, 2),
                    "algorithmic_flop_per_launch": flops[dom]}
    else:
        log(f"[bench] {opc_path} missing: roofline omitted")

    cpu = None
    if args.cpu_sample > 0:
        log(f"[bench] cpu baseline: oracle on {args.cpu_sample} rays ...")
        cpu = cpu_baseline(job, args.cpu_sample)
        log(f"[bench] cpu baseline {cpu['value']:.4f} Mrays/s on {cpu['cores']} threads")

    out = {
        "metric": "Mrays/s fwd+bwd at K=20, batched vs per-call; p50/p99 render latency",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": job.name, "kernels": N, "channels": C, "height": H, "width": W, "K": K,
                   "eta": job.eta, "rays_per_step": rays, "mode": "per-call forward+backward"},
        "latency_ms": {"p50": round(float(np.percentile(per_step, 50)), 5),
                       "p99": round(float(np.percentile(per_step, 99)), 5)},
        "phases_us": {k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in phases.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def R_kb(K: int) -> int:
    for kb in (8, 16, 20, 32, 64):
        if K <= kb:
            return kb
    return 64


if __name__ == "__main__":
    main()
