"""Benchmark of the Diffusion Restore chain step on one MI355X.

Default workload: the real-time loop on the procedural interior (a closed
room of 2,048,020 triangles: instanced noise-displaced meshes, two ceiling
quad lights and one partly occluded light), 1920x1080 frame buffer, path
length <= 8 (d = 28), 4,194,304 chains resident in HBM, FP32, scores from the
reverse-mode adjoint, the camera moving along a 60-frame path.

One timed step of this benchmark is one displayed frame of that loop: the
camera changes (a scene change), so the frame re-initialises every chain
(Alg. 4.1), runs as many evolve steps as a 33.3 ms frame leaves room for
(at least one), and resolves the image (Alg. 4.3); the frame is one captured
HIP graph, replayed once per frame.  `value` = chains x evolve steps per
frame x frames / wall time of the timed frames (chain-steps/s; the
initialise pass, which also evaluates f and the score of every chain, is not
counted as a step).  Also reported: the steady-state evolve rate of the same
chains, the plain multi-kernel form on the same workload, MRSE of the frame
images along the camera path against path-traced references with their own
noise subtracted (split halves), the same loop at 1,048,576 chains, equal-time
path tracing, the roofline of the dominant kernel, and the oracle on the
host's cores.  The procedural 53k-triangle scene (512x512, 65,536 chains) is
reported beside it as a secondary line.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed frames of the real-time loop (secondary lines: evolve steps)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain", action="store_true",
                    help="with --profile-only: the plain multi-kernel form instead of the fused one")
    ap.add_argument("--no-mrse", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 53k-triangle secondary line and the 1,048,576-chain loop")
    ap.add_argument("--no-scaling", action="store_true",
                    help="skip the larger chain counts reported beside the 53k-triangle line")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="skip the launch autotuner (default launch rule)")
    ap.add_argument("--chains", type=int, default=None,
                    help="chains of the measured workload (default: the workload's own count)")
    ap.add_argument("--steps-per-frame", type=int, default=8,
                    help="53k-triangle line and --config: evolve steps per launch")
    ap.add_argument("--frame-steps", type=int, default=None,
                    help="real-time loop: evolve steps per frame (default: as many as fit 33.3 ms, at least 1)")
    ap.add_argument("--profile-only", action="store_true",
                    help="only run warmup + steps launches of the measured workload's dominant kernel (for "
                         "hardware-counter runs; with --config, that configuration's fused launches)")
    ap.add_argument("--headline-spheres", action="store_true",
                    help="print the 53k-triangle line (512x512, 65,536 chains) as the main line instead")
    ap.add_argument("--config", default=None,
                    help="measure a named larger configuration (instances, spheres_1080p_L16, spheres_specular); "
                         "prints its own JSON line")
    ap.add_argument("--config-chains", type=int, default=None,
                    help="with --config: run the configuration with this many chains instead of its own")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--traffic-summary", nargs="+", metavar="DIR",
                    help="no GPU: write the HBM traffic summary of the dominant kernel from rocprofv3 --pmc "
                         "output folders: FETCH_SIZE and WRITE_SIZE of --profile-only, then of --copy-probe, "
                         "optionally followed by TCC_HIT_sum/TCC_MISS_sum and SQ_WAVE_CYCLES/SQ_ACTIVE_INST_VALU "
                         "folders (with --headline-spheres: the 53k-triangle kernel)")
    return ap.parse_args()


# ---- HBM traffic of the dominant kernel, from hardware counters.  Each
# summary records a digest of the kernel sources and the launch shape; a bench
# run whose sources or shape differ reports traffic as null.
TRAFFIC_FILES = {
    "interior": os.path.join(ROOT, "profiles", "k_step_fused_interior2M_4Mchains_traffic.txt"),
    "spheres": os.path.join(ROOT, "profiles", "k_step_fused_spheres53k_traffic.txt"),
}
TRAFFIC_TITLES = {
    "interior": "k_step_fused<8, false>: procedural interior 2,048,020 triangles, 1920x1080, L = 8, one lane per chain",
    "spheres": "k_step_fused_pair<8, false>: procedural spheres 53k triangles, 512x512, L = 8",
}
KERNEL_SOURCES = ["paper_2605_08916_amd/csrc/dr_lib.hip", "paper_2605_08916_amd/csrc/dr_kernels.h",
                  "paper_2605_08916_amd/csrc/dr_device.h", "paper_2605_08916_amd/csrc/dr_adjoint.h",
                  "paper_2605_08916_amd/csrc/dr_chain.h", "paper_2605_08916_amd/csrc/dr_machine.h",
                  "paper_2605_08916_amd/csrc/bvh_build.cpp", "include/dr.h", "paper_2605_08916_amd/build.py"] + [
                  f"paper_2605_08916_amd/csrc/dr_inst_{x}.hip" for x in "abcde"]


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _pmc_rows(folder, counter):
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"no {counter} rows under {folder}")
    return rows


def write_traffic_summary(dirs, workload, chains, per_launch, cmd):
    fetch_dir, write_dir, cfetch_dir, cwrite_dir = dirs[:4]

    def fused_mean(folder, counter, kernel="k_step_fused"):
        v = [x for k, x in _pmc_rows(folder, counter) if kernel in k]
        if not v:
            raise SystemExit(f"no {kernel} dispatch with {counter} under {folder}")
        return sum(v) / len(v), len(v)

    def copy_kib(folder, counter):
        return max(x for k, x in _pmc_rows(folder, counter) if "copyBuffer" in k)

    fk, nf = fused_mean(fetch_dir, "FETCH_SIZE")
    wk, nw = fused_mean(write_dir, "WRITE_SIZE")
    copy_bytes = 4 * (1 << 28)
    fs = copy_bytes / (copy_kib(cfetch_dir, "FETCH_SIZE") * 1024.0)
    ws = copy_bytes / (copy_kib(cwrite_dir, "WRITE_SIZE") * 1024.0)
    rd, wr = fk * 1024.0 * fs, wk * 1024.0 * ws
    lines = [
        f"# HBM traffic of {TRAFFIC_TITLES[workload]}",
        f"# counters: rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -d <out> -- {cmd}",
        "# calibration: rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -d <out> -- python3 bench.py --copy-probe",
        "# written by: python3 bench.py --traffic-summary <fetch> <write> <copy_fetch> <copy_write> [<tcc> <sq2>]"
        + (" --headline-spheres" if workload == "spheres" else ""),
        "# tcc: --pmc TCC_HIT_sum TCC_MISS_sum; sq2: --pmc SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_ACTIVE_INST_ANY "
        "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_VMEM SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_SCA SQ_INST_CYCLES_VMEM_RD "
        "(same --profile-only command); valu_issue_frac is per wavefront",
        f"sources_digest: {sources_digest()}",
        f"chains: {chains}",
        f"steps_per_launch: {per_launch}",
        f"dispatches_fetch: {nf}",
        f"dispatches_write: {nw}",
        f"fetch_kib_per_dispatch: {fk:.1f}",
        f"write_kib_per_dispatch: {wk:.1f}",
        f"copy_fetch_scale: {fs:.4f}",
        f"copy_write_scale: {ws:.4f}",
        f"hbm_read_bytes_per_launch: {rd:.0f}",
        f"hbm_write_bytes_per_launch: {wr:.0f}",
        f"hbm_bytes_per_launch: {rd + wr:.0f}",
        f"hbm_bytes_per_chain_step: {(rd + wr) / (chains * per_launch):.1f}",
    ]
    if len(dirs) >= 6:
        hit, _ = fused_mean(dirs[4], "TCC_HIT_sum")
        miss, _ = fused_mean(dirs[4], "TCC_MISS_sum")
        valu, _ = fused_mean(dirs[5], "SQ_ACTIVE_INST_VALU")
        wc, _ = fused_mean(dirs[5], "SQ_WAVE_CYCLES")
        wait, _ = fused_mean(dirs[5], "SQ_WAIT_ANY")
        lines += [f"l2_hit_rate: {hit / (hit + miss):.4f}", f"valu_issue_frac: {valu / wc:.4f}",
                  f"wait_frac: {wait / wc:.4f}"]
    if workload == "interior":
        # the frame's other full path evaluation: the re-initialisation kernel
        fi, _ = fused_mean(fetch_dir, "FETCH_SIZE", "k_init_eval")
        wi, _ = fused_mean(write_dir, "WRITE_SIZE", "k_init_eval")
        lines += [f"init_eval_hbm_read_bytes_per_launch: {fi * 1024.0 * fs:.0f}",
                  f"init_eval_hbm_write_bytes_per_launch: {wi * 1024.0 * ws:.0f}"]
        if len(dirs) >= 6:
            hit, _ = fused_mean(dirs[4], "TCC_HIT_sum", "k_init_eval")
            miss, _ = fused_mean(dirs[4], "TCC_MISS_sum", "k_init_eval")
            valu, _ = fused_mean(dirs[5], "SQ_ACTIVE_INST_VALU", "k_init_eval")
            wc, _ = fused_mean(dirs[5], "SQ_WAVE_CYCLES", "k_init_eval")
            wait, _ = fused_mean(dirs[5], "SQ_WAIT_ANY", "k_init_eval")
            lines += [f"init_eval_l2_hit_rate: {hit / (hit + miss):.4f}", f"init_eval_valu_issue_frac: {valu / wc:.4f}",
                      f"init_eval_wait_frac: {wait / wc:.4f}"]
    with open(TRAFFIC_FILES[workload], "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _traffic_kv(workload, chains, per_launch):
    """The committed counter summary of the workload's dominant kernel, or {}
    when it is missing, was taken on another launch shape, or the kernel
    sources changed since."""
    try:
        with open(TRAFFIC_FILES[workload]) as f:
            kv = dict(l.split(": ", 1) for l in f.read().splitlines() if l and not l.startswith("#"))
    except OSError:
        return {}
    if (kv.get("sources_digest") != sources_digest() or int(kv.get("chains", -1)) != chains
            or int(kv.get("steps_per_launch", -1)) != per_launch):
        return {}
    return kv


def read_counters(workload, chains, per_launch):
    """L2 hit rate and VALU issue fraction from the counter summary."""
    kv = _traffic_kv(workload, chains, per_launch)
    return {k: float(kv[k]) for k in ("l2_hit_rate", "valu_issue_frac") if k in kv}


def read_traffic(workload, chains, per_launch):
    """HBM bytes per launch from the counter summary, or None."""
    kv = _traffic_kv(workload, chains, per_launch)
    return float(kv["hbm_bytes_per_launch"]) if "hbm_bytes_per_launch" in kv else None


def alg_bytes_per_chain_step(rays, nodes, tris, d, L):
    """Algorithmic bytes per chain-step of the fused kernel: state x and score
    read+write, killed flag read+write, path record write+read, 4-wide BVH
    nodes (128 B per visit) and triangles (48 B per test) fetched by
    traversal, the material/light records per vertex, and the 3-channel
    splat read-modify-write."""
    verts = rays / 2.0
    b_state = 16 * d + 8 + 8 * (L - 1)
    b_trav = nodes * 128 + tris * 48
    b_shade = verts * (48 + 48 + 80)
    b_splat = 24
    return b_state + b_trav + b_shade + b_splat


def traversal_work(ch, warm=3, n=4):
    """Rays, node visits, triangle tests and adjoint fraction per chain-step
    from the library's counters (a separate, untimed pass)."""
    for _ in range(warm):
        ch.step(1)
    ch.set_counters(True)
    b0 = ch.stats()
    ch.step(n)
    b1 = ch.stats()
    ch.set_counters(False)
    cs = b1["chain_steps"] - b0["chain_steps"]
    return tuple((b1[k] - b0[k]) / cs for k in ("rays", "node_visits", "tri_tests", "adjoints"))


def chain_count_scaling(torch, dr, scene, L, F, hbm_copy, counts=(262144, 1048576)):
    """The same scene and step at larger chain counts (the default launch rule
    picks one lane per chain there): chain-steps/s and the algorithmic
    bandwidth against the plain-copy bandwidth.  More resident wavefronts hide
    more of the traversal's fetch latency."""
    d = 4 * (L - 1)
    out = []
    for n in counts:
        ch = dr.Chains(scene, n, L, 4048, mode=dr.DR_MODE_FUSED)
        ms, _, _ = time_steps(ch, torch, 4 * F, F, F)
        ms_launch = time_kernel_only(ch, torch, 3, F)
        rays, nodes, tris, _ = traversal_work(ch, warm=0, n=2)
        b = alg_bytes_per_chain_step(rays, nodes, tris, d, L)
        gbs = b * n * F / (ms_launch * 1e-3) / 1e9
        out.append({"chains": n, "value": n / (ms * 1e-3), "ms_per_step": ms, "lanes_per_chain":
                    ch.get_launch()["lanes_per_chain"], "alg_GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
                    "frac_of_achievable": gbs / hbm_copy})
        ch.close()
    return out


def lum(img):
    return 0.2126 * img[0] + 0.7152 * img[1] + 0.0722 * img[2]


def mrse(img, ref):
    return float((((img - ref) ** 2) / (ref ** 2 + 1e-2)).mean())


def time_steps(ch, torch, steps, warmup, per_frame=1):
    """Average ms per evolve step, steps issued as frames of dr_step(per_frame)
    + dr_resolve, with events on the launch stream; also the median over the
    frames of ms per step."""
    stream = torch.cuda.current_stream()
    out = torch.empty((3, ch.scene.W * ch.scene.H), device="cuda", dtype=torch.float32)
    frames = max(1, steps // per_frame)
    for _ in range(max(1, warmup // per_frame)):
        ch.step(per_frame)
        ch.resolve(out)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(frames + 1)]
    ev[0].record(stream)
    for i in range(frames):
        ch.step(per_frame)
        ch.resolve(out)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) / per_frame for i in range(frames)]
    return ev[0].elapsed_time(ev[frames]) / (frames * per_frame), frames * per_frame, float(np.median(per))


def achievable_bandwidth(torch, reps=5):
    """HBM bandwidth a plain device copy reaches on this GPU (1 GiB read + 1
    GiB written per copy), GB/s."""
    n = 1 << 28
    src = torch.ones(n, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def frame_mrse(ch, torch, ms_per_step, ref, frame_ms=33.3):
    """MRSE of the image one frame of frame_ms gives: re-initialise (a scene
    change), as many steps as fit, resolve."""
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ch.reinit(1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_init = e0.elapsed_time(e1)
    n = max(1, int((frame_ms - ms_init) / ms_per_step))
    e0.record(stream)
    ch.reinit(1)
    ch.step(n)
    ch.resolve()
    e1.record(stream)
    torch.cuda.synchronize()
    img, _ = ch.image_read()
    return dict(steps=n, frame_ms=e0.elapsed_time(e1), init_ms=ms_init, mrse=mrse(img.astype(np.float64), ref))


def time_kernel_only(ch, torch, launches, per_launch):
    """Average ms of one evolve launch dr_step(per_launch) (events bracket each
    launch; the launch is the queue reset fill plus the persistent kernel)."""
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(launches)]
    for a, b in evs:
        a.record(stream)
        ch.step(per_launch)
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


def host_threads():
    """Threads for the oracle: the CPUs this process may run on (at most 16,
    the host share a one-GPU job gets on the GPU machines), and what nproc
    reports."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail)), avail, os.cpu_count() or 1


def cpu_baseline(sc, L, seconds, k0, n=256, label="the same scene and parameters"):
    """The oracle as it stands on this host's cores, on a bounded sample of the
    same workload: a subset of the chains for a few steps."""
    import oracle
    nthreads, avail, nproc = host_threads()
    S = oracle.Scene(sc)
    C = oracle.Chains.scene(S, L, n, seed=1, k0=k0)
    C.init(nthreads=nthreads)
    t0 = time.perf_counter()
    C.step(2, nthreads=nthreads)
    per = (time.perf_counter() - t0) / (2 * n)
    steps = max(2, int(seconds / max(per * n, 1e-9)))
    t0 = time.perf_counter()
    C.step(steps, nthreads=nthreads)
    dt = time.perf_counter() - t0
    return dict(value=n * steps / dt, unit="chain-steps/s", cores=nthreads, kind="oracle",
                sample=f"{n} chains x {steps} evolve steps of {label} (FP64 oracle, {dt:.1f} s, "
                       f"{nthreads} threads; {avail} CPUs available to the process, nproc {nproc})",
                host_cpus_available=avail, nproc=nproc)


def run_config(a, torch, dr, inputs):
    """One JSON line for a larger configuration: chain-steps/s in frames of F
    steps, rays and traversal work per chain-step, and the image a 33.3 ms
    frame gives (re-initialise + steps + resolve) against independent path
    tracing at 64 spp.  The interior configuration runs the real-time loop: a
    captured frame graph replayed along the camera path, one reference per
    sampled frame."""
    fac, L, N = inputs.CONFIGS[a.config]
    if a.config_chains:
        N = a.config_chains
    sc = fac()
    d = 4 * (L - 1)
    scene = dr.Scene(sc)
    sigma = None
    if a.config == "spheres_1080p_L16":
        sigma = torch.from_numpy(inputs.per_chain_sigma(d, N, seed=4)).cuda()
    F = max(1, a.steps_per_frame)
    ch = dr.Chains(scene, N, L, 2024, sigma=sigma)
    ms, steps, med = time_steps(ch, torch, a.steps, a.warmup, F)
    ch.set_counters(True)
    b0 = ch.stats()
    ch.step(2)
    b1 = ch.stats()
    ch.set_counters(False)
    cs = b1["chain_steps"] - b0["chain_steps"]
    rays = (b1["rays"] - b0["rays"]) / cs
    res = {"metric": "chain-steps/s (f+grad log f), larger configuration", "value": N / (ms * 1e-3),
           "unit": "chain-steps/s", "ms_per_step": ms, "ms_per_step_median_frame": med, "steps": steps,
           "config": {"workload": a.config, "triangles": int(sc["indices"].shape[0]), "width": scene.W,
                      "height": scene.H, "path_len": L, "chains": N, "per_chain_sigma": sigma is not None,
                      "steps_per_frame": F, "launch": ch.get_launch(), "scene": scene.stats()},
           "rays_per_s": rays * N / (ms * 1e-3),
           "per_chain_step": {"rays": rays, "node_visits": (b1["node_visits"] - b0["node_visits"]) / cs,
                              "tri_tests": (b1["tri_tests"] - b0["tri_tests"]) / cs,
                              "adjoint_fraction": (b1["adjoints"] - b0["adjoints"]) / cs}}
    if not a.no_mrse:
        if a.config == "interior":
            # frame graph: re-init + n steps + resolve, replayed along the camera path
            stream = torch.cuda.Stream()
            img = torch.zeros((3, scene.W * scene.H), device="cuda")
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ch.reinit(1)
            torch.cuda.synchronize()
            e0.record()
            ch.reinit(2)
            e1.record()
            torch.cuda.synchronize()
            reinit_ms = e0.elapsed_time(e1)
            # as many steps as fit the 33.3 ms frame after the re-initialisation
            # (1 ms kept for the resolve); at least one
            n = max(1, int((33.3 - 1.0 - reinit_ms) / ms))
            with torch.cuda.stream(stream):
                frame = ch.capture_frame(n, True, img, stream)
            frames = []
            for f in (0, 20, 40, 59):
                cam = inputs.camera_path(sc, f)
                scene.set_camera(cam)
                e0.record(stream)
                frame.launch(stream)
                e1.record(stream)
                stream.synchronize()
                ref = scene.pt_render(L, 700 + f, 64)
                torch.cuda.synchronize()
                frames.append({"frame": f, "frame_ms": e0.elapsed_time(e1),
                               "mrse": mrse(img.cpu().numpy().astype(np.float64),
                                            ref.cpu().numpy().astype(np.float64))})
            frame.close()
            res["realtime_loop"] = {"steps_per_frame": n, "reinit_ms": reinit_ms, "frames": frames,
                                    "reference": "independent path tracing, 64 spp per pixel"}
        else:
            ref = scene.pt_render(L, 777, 64)
            torch.cuda.synchronize()
            res["mrse_33ms"] = dict(frame_mrse(ch, torch, ms, ref.cpu().numpy().astype(np.float64)),
                                    reference="independent path tracing, 64 spp per pixel")
    print(json.dumps(res))


def mrse_split(img, r1, r2):
    """MRSE of img against the mean R of two independent path-traced
    references r1, r2, with the references' own noise subtracted: the
    expected squared difference of img and R is img's own error plus var(R),
    and (r1 - r2)/2 has exactly var(R) as its expected square (split
    halves).  Returns (corrected, raw, reference-noise term)."""
    R = 0.5 * (r1 + r2)
    den = R ** 2 + 1e-2
    raw = float((((img - R) ** 2) / den).mean())
    noise = float(((0.25 * (r1 - r2) ** 2) / den).mean())
    return raw - noise, raw, noise


class Refs:
    """Split-half path-traced references of frames of the camera path,
    rendered once and shared by every loop that is scored."""

    def __init__(self, torch, scene, sc, L, spp, cams):
        self.torch, self.scene, self.sc, self.L, self.spp, self.cams = torch, scene, sc, L, spp, cams
        self.cache = {}

    def get(self, f):
        if f not in self.cache:
            self.scene.set_camera(self.cams[f])
            r1 = self.scene.pt_render(self.L, 100000 + f, self.spp)
            r2 = self.scene.pt_render(self.L, 200000 + f, self.spp)
            self.torch.cuda.synchronize()
            self.cache[f] = (r1.cpu().numpy().astype(np.float64), r2.cpu().numpy().astype(np.float64))
        return self.cache[f]


def realtime_loop(torch, dr, scene, cams, N, L, K, W, mode, frame_steps=None, refs=None, mrse_frames=(),
                  seed=2024, budget_ms=33.3, tune=True, init_refill=None):
    """The real-time loop: one captured frame graph (re-initialise for the
    new camera, n evolve steps, resolve), replayed once per displayed frame
    along the camera path.  n = frame_steps, or as many steps as fit the
    frame budget after the re-initialisation and the resolve (at least 1).
    Everything runs on one stream of its own (the library calls take torch's
    current stream).  init_refill (1 on, 2 off) sets the initialise pass's
    form before the autotuner (which may change it) runs."""
    stream = torch.cuda.Stream()
    img = torch.zeros((3, scene.W * scene.H), device="cuda", dtype=torch.float32)
    scene.set_camera(cams[0])
    tuned = None
    with torch.cuda.stream(stream):
        ch = dr.Chains(scene, N, L, seed, mode=mode)
        if init_refill:
            ch.set_launch(init_refill=init_refill)
        if tune and mode == dr.DR_MODE_FUSED:
            # the launch autotuner on the live chains (they are re-initialised next)
            from paper_2605_08916_amd import autotune
            t = autotune.tune(ch, reps=2, use_cache=False, per_launch=frame_steps or 1, restore=False,
                              keep_within=0.03)
            ti = autotune.tune_init(ch)
            tuned = {"cfg": t["cfg"], "ms_per_step": t["ms"], "default_ms_per_step": t["current_ms"],
                     "candidates": len(t["sweep"]), "init_ms": ti}
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        for rep in range(2):  # the second pass is the calibration
            ev[0].record(stream)
            ch.reinit(1 + rep)
            ev[1].record(stream)
            ch.step(1)
            ev[2].record(stream)
            ch.resolve(img)
            ev[3].record(stream)
            stream.synchronize()
        reinit_ms, step_ms, resolve_ms = (ev[i].elapsed_time(ev[i + 1]) for i in range(3))
        n = frame_steps if frame_steps is not None else max(1, int((budget_ms - reinit_ms - resolve_ms) / step_ms))
        frame = ch.capture_frame(n, True, img, stream)
    for i in range(W):
        scene.set_camera(cams[i % len(cams)])
        frame.launch(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    t0 = time.perf_counter()
    for i in range(K):
        scene.set_camera(cams[(W + i) % len(cams)])   # waits for the frame in flight
        evs[i][0].record(stream)
        frame.launch(stream)
        evs[i][1].record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fms = [x.elapsed_time(y) for x, y in evs]
    out = {"chains": N, "steps_per_frame": n, "frames": K, "wall_s": wall,
           "ms_per_frame": wall * 1e3 / K, "gpu_ms_per_frame_median": float(np.median(fms)),
           "gpu_ms_per_frame_max": float(np.max(fms)),
           "chain_steps_per_s": N * n * K / wall, "evaluations_per_s": N * (n + 1) * K / wall,
           "calibration_ms": {"reinit": reinit_ms, "step": step_ms, "resolve": resolve_ms},
           "within_budget": bool(np.max(fms) <= budget_ms), "autotune": tuned}
    if refs is not None and mrse_frames:
        per = []
        for f in mrse_frames:
            r1, r2 = refs.get(f)
            scene.set_camera(cams[f])
            frame.launch(stream)
            stream.synchronize()
            im = img.cpu().numpy().astype(np.float64)
            m, raw, noise = mrse_split(im, r1, r2)
            per.append({"frame": f, "mrse": m, "mrse_raw": raw, "reference_noise": noise})
        out["mrse_per_frame"] = per
        out["mrse_mean"] = float(np.mean([p["mrse"] for p in per]))
    frame.close()
    return out, ch, stream


def realtime_line(a, torch, dr, inputs):
    """The default JSON line: the real-time loop on the 2M-triangle interior
    at 1920x1080 with 4,194,304 chains."""
    fac, L, N_def = inputs.CONFIGS["interior"]
    N = a.chains or a.config_chains or N_def
    d = 4 * (L - 1)
    sc = fac()
    scene = dr.Scene(sc)
    cams = [inputs.camera_path(sc, f) for f in range(60)]
    K, W = max(1, a.steps), max(0, a.warmup)
    mrse_frames = [] if a.no_mrse else list(range(0, 60, 4)) + [59]
    refs = None if a.no_mrse else Refs(torch, scene, sc, L, 32, cams)

    rt, ch, stream = realtime_loop(torch, dr, scene, cams, N, L, K, W, dr.DR_MODE_FUSED, a.frame_steps, refs,
                                   mrse_frames, tune=not a.no_tune)
    n = rt["steps_per_frame"]
    # steady-state evolve rate of the same chains (no re-initialisation):
    # frames of 4 steps + resolve
    scene.set_camera(cams[0])
    with torch.cuda.stream(stream):
        ch.reinit(3)
        ms_ss, _, _ = time_steps(ch, torch, 12, 4, 4)
        # the dominant kernel: the evolve launch of the frame, n steps per launch
        ms_launch = time_kernel_only(ch, torch, 3, n)
        # counters pass (not timed): rays and traversal work per chain-step
        rays, nodes, tris, adj = traversal_work(ch, warm=0, n=1)
        launch_cfg = ch.get_launch()
        k0 = ch.read_state()["k0"]
    torch.cuda.synchronize()
    ch.close()

    bytes_step = alg_bytes_per_chain_step(rays, nodes, tris, d, L)
    achieved = bytes_step * N * n / (ms_launch * 1e-3) / 1e9
    traffic = read_traffic("interior", N, n)
    counters = read_counters("interior", N, n)
    hbm_copy = achievable_bandwidth(torch)
    res = {
        "metric": "chain-steps/s (f+∇log f) and MRSE at 33 ms/frame, fused vs plain",
        "value": rt["chain_steps_per_s"],
        "unit": "chain-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": rt["ms_per_frame"],
        "step_is": "one displayed frame of the real-time loop: re-initialise (camera change) + "
                   f"{n} evolve step(s) + resolve, one captured HIP graph",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "realtime_loop_procedural_interior_2M_tris_1920x1080_L8_d28_4194304chains",
                   "triangles": int(sc["indices"].shape[0]), "width": scene.W, "height": scene.H, "path_len": L,
                   "chains": N, "stddev": 5e-3, "dt": 1e-5, "gamma": 0.5, "m": 64, "form": "fused",
                   "frame_budget_ms": 33.3, "camera_path_frames": 60, "launch": launch_cfg,
                   "scene": scene.stats()},
        "realtime": rt,
        "steady_state_evolve": {"value": N / (ms_ss * 1e-3), "ms_per_step": ms_ss,
                                "issue": "frames of dr_step(4) + resolve, no re-initialisation"},
        "rays_per_s": rays * rt["chain_steps_per_s"],
        "per_chain_step": {"rays": rays, "node_visits": nodes, "tri_tests": tris, "adjoint_fraction": adj,
                           "alg_bytes": bytes_step},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "hbm_measured_GBs": None if traffic is None else traffic / (ms_launch * 1e-3) / 1e9,
                     "achievable_copy_GBs": hbm_copy, "frac_of_achievable": achieved / hbm_copy,
                     "l2_hit_rate": counters.get("l2_hit_rate"), "valu_issue_frac": counters.get("valu_issue_frac"),
                     "alg_bytes_per_launch": bytes_step * N * n,
                     "kernel": f"k_step_fused{'_pair' if launch_cfg['lanes_per_chain'] == 2 else ''}<{L}, false>",
                     "launch_ms": ms_launch, "steps_per_launch": n,
                     "note": "achieved = algorithmic bytes / launch time; most node and triangle bytes are "
                             "served by the L2 and the MALL, hbm_measured_GBs is what reaches HBM"},
    }
    # ---- plain multi-kernel form: the same frames with the same step count
    # (identical decisions from identical streams, so the same image: the
    # frame-time ratio is the speed ratio at equal MRSE)
    if not a.no_plain:
        # the same initialise form as the fused loop: the frames differ only in the steps
        irf = (rt.get("autotune") or {}).get("init_ms", {}).get("init_refill")
        pr, cp, _ = realtime_loop(torch, dr, scene, cams, N, L, min(K, 4), 1, dr.DR_MODE_PLAIN, n, refs,
                                  mrse_frames[:2], init_refill=irf)
        cp.close()
        res["plain"] = pr
        res["fused_over_plain"] = pr["ms_per_frame"] / rt["ms_per_frame"]
    # ---- equal-time path tracing: the samples per pixel that fit 33.3 ms
    if refs is not None:
        scene.set_camera(cams[0])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        scene.pt_render(L, 5, 1)
        e0.record()
        scene.pt_render(L, 5, 1)
        e1.record()
        torch.cuda.synchronize()
        spp = max(1, int(33.3 / e0.elapsed_time(e1)))
        pm = []
        for f in mrse_frames[:4]:
            scene.set_camera(cams[f])
            e0.record()
            im = scene.pt_render(L, 900 + f, spp)
            e1.record()
            torch.cuda.synchronize()
            r1, r2 = refs.get(f)
            pm.append({"frame": f, "mrse": mrse_split(im.cpu().numpy().astype(np.float64), r1, r2)[0],
                       "frame_ms": e0.elapsed_time(e1)})
        res["pt_equal_time_33ms"] = {"spp": spp, "frames": pm, "mrse_mean": float(np.mean([p["mrse"] for p in pm]))}
        res["mrse_reference"] = ("independent path tracing, two 32-spp halves per frame (seeds 100000+f, "
                                 "200000+f); MRSE against their mean minus the halves' own noise")
        # ---- a static view (frame 0): MRSE after 1, 4, 16 and 64 evolve steps
        # from one re-initialisation, at 1,048,576 and at N chains: how the
        # image error falls with steps and with chains once the start-up
        # bias of a fresh initialisation has decayed
        scene.set_camera(cams[0])
        r1, r2 = refs.get(0)
        # a second, 8x larger reference of the same frame (two 256-spp halves):
        # the MRSE against it shows how much of the figure is reference noise
        h1 = scene.pt_render(L, 300000, 256).cpu().numpy().astype(np.float64)
        h2 = scene.pt_render(L, 400000, 256).cpu().numpy().astype(np.float64)
        conv = {}
        for n_ch in sorted({1 << 20, N}):
            cc = dr.Chains(scene, n_ch, L, 77, mode=dr.DR_MODE_FUSED)
            cc.set_launch(**{k: v for k, v in launch_cfg.items() if k in ("block", "blocks_per_cu", "grab",
                                                                          "lanes_per_chain")})
            img0 = torch.zeros((3, scene.W * scene.H), device="cuda", dtype=torch.float32)
            cc.reinit(1)
            done, rows = 0, []
            t_ms = 0.0
            for total in (1, 4, 16, 64):
                e0.record()
                cc.step(total - done)
                e1.record()
                torch.cuda.synchronize()
                t_ms += e0.elapsed_time(e1)
                done = total
                cc.resolve(img0)
                im0 = img0.cpu().numpy().astype(np.float64)
                rows.append({"steps": total, "mrse": mrse_split(im0, r1, r2)[0],
                             "mrse_ref256": mrse_split(im0, h1, h2)[0], "step_ms_total": t_ms})
            cc.close()
            conv[str(n_ch)] = rows
        res["static_view_convergence"] = {"frame": 0, "by_chains": conv,
                                          "reference": "mrse: two 32-spp halves; mrse_ref256: two 256-spp halves"}
    # ---- the same loop with 1,048,576 chains (one GPU's share at 4 GPUs) and
    # with one chain per pixel (the paper's dispatch size, Sec. 6)
    if not a.no_secondary and N > (1 << 20):
        r1m, c1, _ = realtime_loop(torch, dr, scene, cams, 1 << 20, L, min(K, 10), 2, dr.DR_MODE_FUSED, None, refs,
                                   mrse_frames, tune=not a.no_tune)
        c1.close()
        res["realtime_1M_chains"] = r1m
        npx = scene.W * scene.H
        if npx < N:
            rpx, cpx, _ = realtime_loop(torch, dr, scene, cams, npx, L, min(K, 10), 2, dr.DR_MODE_FUSED, None, refs,
                                        mrse_frames, tune=not a.no_tune)
            cpx.close()
            res["realtime_one_chain_per_pixel"] = rpx
        # the paper's own frame model: one dispatch per frame, the initialise
        # pass alone whenever the camera has moved (Sec. 4.3, Sec. 6)
        rin, cin, _ = realtime_loop(torch, dr, scene, cams, N, L, min(K, 10), 2, dr.DR_MODE_FUSED, 0, refs,
                                    mrse_frames, tune=False)
        cin.close()
        rin["frame_is"] = "initialise pass + resolve: one dispatch per frame, the initialise one after a camera move"
        res["realtime_initialise_only"] = rin
    if not a.no_secondary:
        res["procedural_spheres_53k"] = spheres_line(a, torch, dr, inputs, secondary=True)
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(sc, L, a.cpu_seconds, k0, n=256,
                                           label="the interior scene (2,048,020 triangles, L = 8) with the same "
                                                 "parameters")
    scene.close()
    return res


def spheres_line(a, torch, dr, inputs, secondary=False):
    """The procedural 53k-triangle scene (512x512, L = 8, 65,536 chains):
    evolve steps in frames of F steps + resolve, fused and plain forms; with
    secondary=False the full line (roofline, chain-count scaling, MRSE at
    33 ms, equal-time path tracing, oracle baseline)."""
    sc = inputs.procedural_spheres(seed=1)
    L, N = 8, (a.chains if (a.chains and not secondary) else 65536)
    d = 4 * (L - 1)
    seed = 2024
    scene = dr.Scene(sc)
    F = max(1, a.steps_per_frame)
    steps = max(16, a.steps) if secondary else a.steps
    ch = dr.Chains(scene, N, L, seed, mode=dr.DR_MODE_FUSED)
    torch.cuda.synchronize()
    ms_fused, steps_done, ms_median = time_steps(ch, torch, steps, a.warmup, F)
    value = N / (ms_fused * 1e-3)
    launch_cfg = ch.get_launch()
    rays, nodes, tris, adj = traversal_work(ch, warm=0, n=4)
    out = {"workload": "procedural_spheres_53k_tris_512x512_L8_d28_65536chains", "value": value,
           "unit": "chain-steps/s", "ms_per_step": ms_fused, "steps": steps_done, "steps_per_frame": F,
           "rays_per_s": rays * value, "per_chain_step": {"rays": rays, "node_visits": nodes, "tri_tests": tris,
                                                          "adjoint_fraction": adj}, "launch": launch_cfg}
    if not a.no_plain:
        cp = dr.Chains(scene, N, L, seed, mode=dr.DR_MODE_PLAIN)
        ms_plain, _, _ = time_steps(cp, torch, max(2 * F, steps // 2), a.warmup, F)
        out["plain"] = {"value": N / (ms_plain * 1e-3), "ms_per_step": ms_plain}
        out["fused_over_plain"] = ms_plain / ms_fused
        cp.close()
    if secondary:
        ch.close()
        scene.close()
        return out
    # full line (--headline-spheres)
    ms_single, _, _ = time_steps(ch, torch, max(8, a.steps // 4), 2, 1)
    ms_launch = time_kernel_only(ch, torch, max(4, a.steps // (4 * F)), F)
    k0 = ch.read_state()["k0"]
    bytes_step = alg_bytes_per_chain_step(rays, nodes, tris, d, L)
    achieved = bytes_step * N * F / (ms_launch * 1e-3) / 1e9
    traffic = read_traffic("spheres", N, F)
    counters = read_counters("spheres", N, F)
    hbm_copy = achievable_bandwidth(torch)
    res = {
        "metric": "chain-steps/s (f+∇log f) and MRSE at 33 ms/frame, fused vs plain",
        "value": value, "unit": "chain-steps/s", "n_gpus": 1, "steps": steps_done, "warmup": a.warmup,
        "ms_per_step": ms_fused, "ms_per_step_median_frame": ms_median, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": out["workload"], "triangles": int(sc["indices"].shape[0]), "width": 512,
                   "height": 512, "path_len": L, "chains": N, "stddev": 5e-3, "dt": 1e-5, "gamma": 0.5, "m": 64,
                   "form": "fused", "steps_per_frame": F, "launch": launch_cfg},
        "single_step_dispatch": {"value": N / (ms_single * 1e-3), "ms_per_step": ms_single},
        "rays_per_s": out["rays_per_s"],
        "per_chain_step": dict(out["per_chain_step"], alg_bytes=bytes_step),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "hbm_measured_GBs": None if traffic is None else traffic / (ms_launch * 1e-3) / 1e9,
                     "achievable_copy_GBs": hbm_copy, "frac_of_achievable": achieved / hbm_copy,
                     "l2_hit_rate": counters.get("l2_hit_rate"), "valu_issue_frac": counters.get("valu_issue_frac"),
                     "traffic_unit": "HBM bytes per launch", "alg_bytes_per_launch": bytes_step * N * F,
                     "kernel": f"k_step_fused{'_pair' if launch_cfg['lanes_per_chain'] == 2 else ''}<{L}, false>",
                     "launch_ms": ms_launch, "steps_per_launch": F},
        "chain_count_scaling": [] if a.no_scaling else chain_count_scaling(torch, dr, scene, L, F, hbm_copy),
    }
    for k in ("plain", "fused_over_plain"):
        if k in out:
            res[k] = out[k]
    if not a.no_mrse:
        ref = scene.pt_render(L, 777, 256)
        torch.cuda.synchronize()
        ref = ref.cpu().numpy().astype(np.float64)
        res["mrse_33ms"] = dict(frame_mrse(ch, torch, ms_fused, ref),
                                reference="independent path tracing, 256 spp per pixel (seed 777)")
    ch.close()
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(sc, L, a.cpu_seconds, k0)
    scene.close()
    return res


def main():
    a = parse()
    if a.traffic_summary:
        if a.headline_spheres:
            n = a.chains or 65536
            F = max(1, a.steps_per_frame)
            cmd = (f"python3 bench.py --headline-spheres --profile-only --steps 8 --warmup 2 --chains {n} "
                   f"--steps-per-frame {F}")
            write_traffic_summary(a.traffic_summary, "spheres", n, F, cmd)
        else:
            n = a.chains or (1 << 22)
            F = a.frame_steps or 1
            cmd = f"python3 bench.py --profile-only --steps 4 --warmup 1 --frame-steps {F}"
            write_traffic_summary(a.traffic_summary, "interior", n, F, cmd)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the chain step has no multi-GPU path in this "
              "build", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2605_08916_amd import dr, inputs

    torch.cuda.set_device(0)
    if a.copy_probe:
        n = 1 << 28
        src = torch.ones(n, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n}))
        return
    if a.profile_only:
        if a.config:
            fac, L, N = inputs.CONFIGS[a.config]
            N = a.config_chains or N
            F = max(1, a.steps_per_frame)
        elif a.headline_spheres:
            fac, L, N = inputs.CONFIGS["spheres"]
            N = a.chains or N
            F = max(1, a.steps_per_frame)
        else:
            fac, L, N = inputs.CONFIGS["interior"]
            N = a.chains or N
            F = a.frame_steps or 1
        sc = fac()
        scene = dr.Scene(sc)
        sigma = None
        if a.config == "spheres_1080p_L16":
            sigma = torch.from_numpy(inputs.per_chain_sigma(4 * (L - 1), N, seed=4)).cuda()
        ch = dr.Chains(scene, N, L, 2024, sigma=sigma, mode=dr.DR_MODE_PLAIN if a.plain else dr.DR_MODE_FUSED)
        if a.config or a.headline_spheres:
            for _ in range(a.warmup + a.steps):
                ch.step(F)
        else:
            # the real-time frame: camera move, re-initialisation, F evolve steps, resolve
            cams = [inputs.camera_path(sc, f) for f in range(60)]
            img = torch.zeros((3, scene.W * scene.H), device="cuda", dtype=torch.float32)
            for i in range(a.warmup + a.steps):
                scene.set_camera(cams[i % len(cams)])
                ch.reinit(1 + i)
                ch.step(F)
                ch.resolve(img)
        torch.cuda.synchronize()
        print(json.dumps({"profile_only_launches": a.warmup + a.steps, "steps_per_launch": F, "chains": N,
                          "config": a.config or ("spheres" if a.headline_spheres else "interior"),
                          "form": "plain" if a.plain else "fused"}))
        return
    if a.config and a.config != "interior":
        run_config(a, torch, dr, inputs)
        return
    if a.headline_spheres:
        print(json.dumps(spheres_line(a, torch, dr, inputs)))
        return
    print(json.dumps(realtime_line(a, torch, dr, inputs)))


if __name__ == "__main__":
    main()
