"""Throughput benchmark of the D3Q19 flux-inlet step on one MI355X.

Default workload: 256^3 pack of overlapping solid spheres (seed 2, radii
uniform in [6, 10], porosity 0.35, six pure-fluid reservoir layers at each z
end), FP32 distributions, BGK tau = 0.8, adaptive flux inlet with Darcy
velocity 1e-4 (Q* = 1e-4 * 256^2), pressure outlet rho = 1.

Prints one JSON line: MLUPS over pore sites for the timed steps, the roofline
of the fused stream-collide kernel (algorithmic bytes per launch over its
mean HIP-event duration), the FP64 CPU oracle timed on a bounded sample of
the same workload, and the learned controller's steps-to-tolerance against
the plain update on a held-out 128^3 pack.

Other workloads (``--config``): pack256h (FP16 deviation storage), pack256m
(MRT collision), pack512 (512^3, porosity 0.25), slit (FP64 16x16x64),
pack384c / pack384ch (the two-fluid colour model on the 384^3 pack, FP32 /
FP16 deviations), pack256c (the colour model on the 256^3 pack) and batch64
(64 samples of uneven size in one batched launch per step, with the
autotuned schedule).

The roofline object carries two byte counts per site: ``bytes_per_lup``,
what this design's step kernels must move (the compact pull table, the
colour model's two passes), and ``bytes_per_lup_survey``, the plain count of
19 populations read and written once plus 18 int32 indices (224 B FP32,
148 B FP16 deviations, 376 B FP64; the colour model adds its two D3Q7
colours and the phase field: 340 B FP32, 208 B FP16), with ``frac`` and
``frac_survey`` the achieved fractions of 8 TB/s under each.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1806_10589_amd", "csrc", f) for f in ("kernels.h", "engine.hip", "pull_format.h")] + [
    os.path.join(ROOT, "paper_1806_10589_amd", "build.py")]  # its compile flags shape the kernels too
COLOUR_SOURCES = KERNEL_SOURCES + [os.path.join(ROOT, "paper_1806_10589_amd", "csrc", "colour.h")]

# Two-fluid pack workload: interfacial tension gamma = 0.01, reached at
# alpha = 0.0156616 (the Laplace law of cylindrical drops on the FP64 oracle,
# tests/golden/colour_calibration.json, written by
# tests/golden/make_colour_calibration.py); contact angle 45 deg through
# phi_solid = -cos(45 deg); unit viscosity ratio (tau = 1, mu = rho0 nu =
# 1/6); capillary number Ca = mu Q* / (gamma eps A) = 1e-5 over the
# 384^2 inlet at porosity eps = 0.30.
ALPHA_GAMMA_001 = 0.0156616
Q_CA_384 = 1e-5 * 0.01 * 0.30 * 384 * 384 / (1.0 / 6.0)

CONFIGS = {
    # name: (builder, lattice kwargs, description)
    "pack256": dict(n=256, porosity=0.35, seed=2, reservoir=6, tau=0.8, darcy=1e-4, precision="fp32"),
    "pack256h": dict(n=256, porosity=0.35, seed=2, reservoir=6, tau=0.8, darcy=1e-4, precision="fp16dev"),
    "pack512": dict(n=512, porosity=0.25, seed=5, reservoir=6, tau=0.8, darcy=1e-5, precision="fp32"),
    "pack256m": dict(n=256, porosity=0.35, seed=2, reservoir=6, tau=0.8, darcy=1e-4, precision="fp32",
                     model="mrt"),
    # two-fluid colour model: non-wetting fluid in the inlet reservoir, wetting elsewhere
    "pack256c": dict(n=256, porosity=0.35, seed=2, reservoir=6, tau=0.8, darcy=1e-4, precision="fp32",
                     model="colour", alpha=0.005, beta=0.7, phi_solid=-0.5),
    # the two-fluid configuration: 384^3 pack, porosity 0.30, gamma 0.01, 45 deg, Ca 1e-5
    "pack384c": dict(n=384, porosity=0.30, seed=3, reservoir=6, tau=1.0, q=Q_CA_384, precision="fp32",
                     model="colour", alpha=ALPHA_GAMMA_001, beta=0.7, phi_solid=-0.7071),
    "pack384ch": dict(n=384, porosity=0.30, seed=3, reservoir=6, tau=1.0, q=Q_CA_384, precision="fp16dev",
                      model="colour", alpha=ALPHA_GAMMA_001, beta=0.7, phi_solid=-0.7071),
    "slit": dict(slit=True, tau=1.0, q=0.5, precision="fp64"),
    # 64 samples of uneven size in one batched launch per step
    "batch64": dict(batch=64, seed=3, edge=(64, 192), porosity=(0.2, 0.45), darcy=(1e-5, 1e-3),
                    reservoir=6, tau=0.8, precision="fp32"),
}
SCHEDULE_CACHE = os.path.join(ROOT, "paper_1806_10589_amd", "schedule_cache.txt")


def bytes_per_lup(precision: str, model: str = "bgk", share8: float = 0.0, share16: float = 0.0,
                  share_run: float = 0.0, share_wide: float = 0.0) -> float:
    """Algorithmic bytes of one pore-site update in this design: 19
    populations read and written once in the storage type, plus the pull
    table: 18 int32 indices, or, on the shares of tiles that read compact
    codes, 18 8-bit or 16-bit codes and the tile's 80-byte header over its
    512 sites; of the 8-bit tiles, the share share_run that the step reads as
    run codes takes 8 bytes per site instead of 18, and 4 more on the share
    share_wide of waves (of all waves) whose list of codes needs a second
    word (not in the colour model's FP16 step, which reads the 8-bit codes).
    The colour model adds, per site: in the phase pass the 7
    colour pairs (A_q, B_q) read (6 of them pulled, with the codes of
    directions 1-6: 2 words of byte codes, 3 of 16-bit codes or 6 int32) and
    N_A + N_B and phi written; in the colour step phi (the neighbours' values
    counted once) and N_A + N_B read and the 7 recoloured pairs written. The
    colours are FP64 in FP64 storage and FP32 otherwise."""
    elem = {"fp64": 8, "fp32": 4, "fp16dev": 2}[precision]
    hdr = 80 / 512
    if precision == "fp16dev" and model == "colour":
        share_run = share_wide = 0.0
    table = (18 * 4 * (1.0 - share8 - share16) + (18 + hdr) * (share8 - share_run) + (8 + hdr) * share_run
             + 4 * share_wide + (36 + hdr) * share16)
    single = 19 * 2 * elem + table
    if model != "colour":
        return single
    ce = 8 if precision == "fp64" else 4
    table6 = 6 * 4 * (1.0 - share8 - share16) + (8 + hdr) * share8 + (12 + hdr) * share16
    return single + (14 * ce + table6 + 2 * ce) + (2 * ce + 14 * ce)


def bytes_per_lup_survey(precision: str, model: str = "bgk") -> float:
    """The plain byte count per site: 19 populations read and written once
    and 18 int32 pull indices; the colour model adds its two D3Q7 colours
    read and written once in the storage type and the phase field once."""
    elem = {"fp64": 8, "fp32": 4, "fp16dev": 2}[precision]
    single = 19 * 2 * elem + 72
    return single if model != "colour" else single + 14 * 2 * elem + 4


PULL_FORMATS = ("run", "compact", "half", "int32")


def pull_share(lats, fmt: str):
    """Set the pull-table format of the lattices; return the shares of their
    tiles that read 8-bit and 16-bit codes, of the tiles whose 8-bit codes
    the single-fluid step reads as run codes, and of the waves (64 sites)
    whose run codes need a second word."""
    from paper_1806_10589_amd import fluxlbm

    code = {"run": fluxlbm.FLBM_PULL_RUN, "compact": fluxlbm.FLBM_PULL_COMPACT, "half": fluxlbm.FLBM_PULL_HALF,
            "int32": fluxlbm.FLBM_PULL_INT32}[fmt]
    t8 = t16 = tr = ww = tiles = 0
    for lat in lats:
        if lat.pull_format()[0] != code:
            lat.set_pull_format(code)
        _, a, b, t = lat.pull_format()
        t8 += a
        t16 += b
        tiles += t
        if fmt == "run":
            r, w = lat.pull_runs()
            tr += r
            ww += w
    return (t8 / tiles, t16 / tiles, tr / tiles, ww / (8 * tiles)) if tiles else (0.0, 0.0, 0.0, 0.0)


def kernel_source_hash(colour: bool = False) -> str:
    import hashlib

    h = hashlib.sha256()
    for path in (COLOUR_SOURCES if colour else KERNEL_SOURCES):
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, precision: str, n_sites: int, pull: str = "compact", colour: bool = False):
    """HBM bytes per step of the step kernel(s) from the committed rocprofv3
    counter summary of this workload, or None when there is none, it was
    taken with another pull-table format, or the kernel sources changed
    since the counters were taken."""
    name = f"k_colour_{workload}_{precision}.md" if colour else f"k_stream_collide_{workload}_{precision}.md"
    path = os.path.join(PROFILE_DIR, name)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256_16") != kernel_source_hash(colour) or vals.get("pull_table", "int32") != pull:
        return None
    try:
        per_site = float(vals["hbm_bytes_per_site"])
    except (KeyError, ValueError):
        return None
    return round(per_site * n_sites)


def make_workload(cfg):
    from paper_1806_10589_amd import inputs

    if cfg.get("slit"):
        mask = inputs.slit_channel(16, 16, 64)
        return mask, dict(tau=cfg["tau"], q_target=cfg["q"], precision=cfg["precision"],
                          periodic_x=False, periodic_y=True), {"porosity": float((mask == 0).mean())}
    mask, phi, nsph = inputs.sphere_pack(cfg["n"], cfg["porosity"], seed=cfg["seed"],
                                         reservoir_layers=cfg["reservoir"])
    q = cfg["q"] if "q" in cfg else cfg["darcy"] * mask.shape[1] * mask.shape[2]
    kw = dict(tau=cfg["tau"], q_target=q, precision=cfg["precision"], periodic_x=True, periodic_y=True,
              model=cfg.get("model", "bgk"))
    for k in ("alpha", "beta", "phi_solid"):
        if k in cfg:
            kw[k] = cfg[k]
    return mask, kw, {"porosity": phi, "spheres": nsph}


def batch_samples(cfg):
    """Seeded batch: edges uniform in [64, 192], porosity uniform in
    [0.2, 0.45], Darcy velocity log-uniform in [1e-5, 1e-3]."""
    import numpy as np

    from paper_1806_10589_amd import inputs

    rng = np.random.default_rng(cfg["seed"])
    out = []
    for i in range(cfg["batch"]):
        n = int(rng.integers(cfg["edge"][0], cfg["edge"][1] + 1))
        phi = float(rng.uniform(*cfg["porosity"]))
        darcy = float(10 ** rng.uniform(np.log10(cfg["darcy"][0]), np.log10(cfg["darcy"][1])))
        mask, ph, _ = inputs.sphere_pack(n, phi, seed=1000 * cfg["seed"] + i, reservoir_layers=cfg["reservoir"])
        out.append((mask, dict(tau=cfg["tau"], q_target=darcy * n * n, precision=cfg["precision"]),
                    dict(edge=n, porosity=ph, darcy=darcy)))
    return out


def run_batch(args, cfg):
    import torch

    from paper_1806_10589_amd import fluxlbm

    t0 = time.perf_counter()
    samples = batch_samples(cfg)
    print(f"[bench] batch of {len(samples)} samples built in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    lats = [fluxlbm.Lattice(m, watchdog_every=1000, **kw) for m, kw, _ in samples]
    n_total = sum(l.n_sites for l in lats)
    share = pull_share(lats, args.pull)
    b = fluxlbm.Batch(lats)
    sched, ms_tuned = b.autotune(SCHEDULE_CACHE if os.access(os.path.dirname(SCHEDULE_CACHE), os.W_OK) else None,
                                 trial_steps=3)
    b.set_schedule(**dict(sched, chunk=100))
    print(f"[bench] schedule {sched} ({ms_tuned:.3f} ms per launch while tuning)", file=sys.stderr, flush=True)
    for l in lats:
        l.init_equilibrium(1.0)
    b.step(args.warmup)
    rc, bad = b.sync()
    if rc != fluxlbm.FLBM_OK:
        raise SystemExit(f"unstable during warm-up (sample {bad})")
    stream = lats[0].stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    b.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    rc, bad = b.sync()
    mlups = n_total * args.steps / (ms_total * 1e-3) / 1e6
    ms_kernel = b.time(args.profile_steps)
    # the same samples stepped one after another by their own launches
    k_seq = max(10, args.steps // 10)
    e0.record(stream)
    for l in lats:
        l.step(k_seq)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_seq = e0.elapsed_time(e1) / k_seq
    bpl = bytes_per_lup(cfg["precision"], "bgk", *share)
    bpl_s = bytes_per_lup_survey(cfg["precision"], "bgk")
    achieved = n_total * bpl / (ms_kernel * 1e-3) / 1e9
    achieved_s = n_total * bpl_s / (ms_kernel * 1e-3) / 1e9
    out = {
        "metric": "MLUPS (pore sites) + HBM GB/s; steps-to-flux-tol, learned vs plain",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_total / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batch64",
            "samples": len(lats),
            "pore_sites": n_total,
            "edges": [x["edge"] for _, _, x in samples],
            "tau": cfg["tau"],
            "precision": cfg["precision"],
            "schedule": sched,
            "pull_table": args.pull,
            "tile_share_8bit_16bit": [round(v, 4) for v in share[:2]],
            "run_share_tiles_waves_wide": [round(v, 4) for v in share[2:]],
        },
        "status": "ok" if rc == fluxlbm.FLBM_OK else f"unstable (sample {bad})",
        "sequential_ms_per_step": round(ms_seq, 5),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "kernel": "k_batch_step",
            "kernel_ms": round(ms_kernel, 5),
            "bytes_per_lup": round(bpl, 2),
            "bytes_per_lup_survey": round(bpl_s, 2),
            "achieved_survey": round(achieved_s, 1),
            "frac_survey": round(achieved_s / HBM_PEAK_GBS, 4),
        },
    }
    m0, kw0, _ = samples[0]
    b.close()
    for l in lats:
        l.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m0, dict(kw0, periodic_x=True, periodic_y=True), args.cpu_steps)
        out["cpu_baseline"]["sample"] = "first sample of the batch: " + out["cpu_baseline"]["sample"]
    print(json.dumps(out), flush=True)


def controller_ab(n=128, margin_frac=0.25, max_steps=None):
    """Steps to |Q_out - Q*| / Q* <= 1e-3 (two-step mean, for good), plain
    update versus the trained controller, on a held-out n^3 pack (porosity
    0.25, seed 5001, tau 0.8, Darcy velocity 1e-5), same GPU; the run goes
    on for margin_frac of the settling time after it. The 512^3 comparison
    takes about 20 minutes (two runs of some 500,000 steps)."""
    from paper_1806_10589_amd import controller

    if not os.path.exists(controller.DEFAULT_WEIGHTS):
        return None
    params, meta = controller.load_weights()
    mask, kw = controller.make_sample(n, 0.25, 5001, tau=0.8, darcy=1e-5)
    if max_steps is None:
        max_steps = max(300000, 4 * n * n)
    progress = (lambda m: print(m, file=sys.stderr, flush=True)) if n > 128 else None
    r = controller.evaluate(params, mask, kw, max_steps=max_steps, settings=controller.settings_of(meta),
                            margin_frac=margin_frac, progress=progress)
    return {"workload": f"pack{n} held out (phi 0.25, seed 5001, tau 0.8, darcy 1e-5), FP32",
            "tol": 1e-3, "margin_frac": margin_frac, "plain_steps": r["plain_steps"],
            "learned_steps": r["learned_steps"], "gain": r.get("gain"),
            "plain_secs": round(r["plain_secs"], 1), "learned_secs": round(r["learned_secs"], 1),
            "controller": list(r["controller"]) if r.get("controller") else None}


def copy_bandwidth(torch, nbytes=2 << 30, reps=20):
    from paper_1806_10589_amd import fluxlbm

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(3):
        fluxlbm.flbm_copy_kernel(a.data_ptr(), b.data_ptr(), nbytes, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fluxlbm.flbm_copy_kernel(a.data_ptr(), b.data_ptr(), nbytes, stream)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(mask, kw, steps, reservoir=6, steps_t1=None):
    """FP64 oracle on the same workload, `steps` steps after one warm-up step
    with every thread OpenMP offers, then `steps_t1` steps on one thread (the
    two-fluid oracle for the colour model, started from the same two-layer
    colour state)."""
    import numpy as np

    import oracle

    colour = kw.get("model") == "colour"
    if colour:
        orc = oracle.OracleColour(mask, tau=kw["tau"], alpha=kw["alpha"], beta=kw["beta"],
                                  phi_solid=kw["phi_solid"], q_target=kw["q_target"],
                                  periodic_x=kw["periodic_x"], periodic_y=kw["periodic_y"])
        na = np.zeros(mask.shape)
        na[:reservoir] = 1.0
        na[mask.astype(bool)] = 0.0
        nb = 1.0 - na
        nb[mask.astype(bool)] = 0.0
        orc.init(na, nb)
        steps = max(1, steps // 4)
    else:
        orc = oracle.OracleLattice(mask, tau=kw["tau"], q_target=kw["q_target"], rho_out=1.0,
                                   periodic_x=kw["periodic_x"], periodic_y=kw["periodic_y"])
        orc.set_mrt(kw.get("model") == "mrt")
        orc.init_equilibrium(1.0)
    threads = oracle.oracle.max_threads()
    orc.step(1, record=False)
    t0 = time.perf_counter()
    orc.step(steps, record=False)
    dt = time.perf_counter() - t0
    n_pore = int((mask == 0).sum())
    out = {
        "value": n_pore * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{steps} steps of the full {mask.shape[2]}x{mask.shape[1]}x{mask.shape[0]} lattice "
                  f"after 1 warm-up step ({dt:.1f} s) on {threads} threads; FP64 dense push-scheme "
                  f"{'two-fluid ' if colour else ''}oracle, OpenMP over z",
        "mlups_per_voxel": mask.size * steps / dt / 1e6,
        "cpu_model": cpu_model(),
        "logical_cpus": os.cpu_count(),
    }
    if steps_t1:
        oracle.oracle.set_threads(1)
        try:
            t0 = time.perf_counter()
            orc.step(steps_t1, record=False)
            dt1 = time.perf_counter() - t0
        finally:
            oracle.oracle.set_threads(threads)
        out["value_1_thread"] = n_pore * steps_t1 / dt1 / 1e6
        out["sample_1_thread"] = f"{steps_t1} steps on 1 thread ({dt1:.1f} s)"
    return out


def roofline_of(config, kw, n, share, ms_kernel, ms_plane, pull):
    """The roofline object of a step: algorithmic bytes of this design and
    the plain survey count, each over the kernels' mean HIP-event duration,
    and the counter traffic of the committed profile when it is current."""
    colour = kw.get("model") == "colour"
    bpl = bytes_per_lup(kw["precision"], kw.get("model", "bgk"), *share)
    bpl_s = bytes_per_lup_survey(kw["precision"], kw.get("model", "bgk"))
    achieved = n * bpl / (ms_kernel * 1e-3) / 1e9
    achieved_s = n * bpl_s / (ms_kernel * 1e-3) / 1e9
    traffic = measured_traffic(config, kw["precision"], n, pull, colour=colour)
    out = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": "k_phase_buf+k_colour_buf" if colour else "k_stream_collide",
        "kernel_ms": round(ms_kernel, 5),
        "plane_kernel_ms": round(ms_plane, 5),
        "bytes_per_lup": round(bpl, 2),
        "bytes_per_lup_survey": round(bpl_s, 2),
        "achieved_survey": round(achieved_s, 1),
        "frac_survey": round(achieved_s / HBM_PEAK_GBS, 4),
    }
    if traffic:
        out["traffic_over_algorithmic"] = round(traffic / (n * bpl), 4)
        out["traffic_gbs"] = round(traffic / (ms_kernel * 1e-3) / 1e9, 1)
    return out


def pack512_line(args, steps=400, warmup=40):
    """Throughput of the same step on the 512^3 pack (porosity 0.25, Darcy
    velocity 1e-5, 35.5M pore sites, FP32, compact pull table): a short
    graph-timed run and the step kernel's HIP-event duration."""
    import torch

    from paper_1806_10589_amd import fluxlbm

    cfg = CONFIGS["pack512"]
    mask, kw, info = make_workload(cfg)
    lat = fluxlbm.Lattice(mask, watchdog_every=1000, **kw)
    try:
        share = pull_share([lat], args.pull)
        lat.init_equilibrium(1.0)
        lat.step(warmup)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(lat.stream)
        lat.step(steps)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ok = lat.sync() == fluxlbm.FLBM_OK
        ms_plane, ms_kernel = lat.profile_kernels(50)
        n = lat.n_sites
        return {"workload": "pack512", "pore_sites": n, "steps": steps, "ms_per_step": round(ms, 5),
                "mlups": round(n / (ms * 1e-3) / 1e6, 1), "status": "ok" if ok else "unstable",
                "porosity": info["porosity"],
                "roofline": roofline_of("pack512", kw, n, share, ms_kernel, ms_plane, args.pull)}
    finally:
        lat.close()
        del lat
        torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", default="pack256", choices=sorted(CONFIGS))
    ap.add_argument("--profile-steps", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--cpu-steps-1-thread", type=int, default=10,
                    help="steps of the oracle timed on one thread after the multi-threaded sample (0: none)")
    ap.add_argument("--no-pack512", action="store_true", help="leave out the 512^3 throughput key")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-controller", action="store_true")
    ap.add_argument("--controller-n", type=int, default=128,
                    help="edge of the held-out pack of the learned-versus-plain comparison "
                         "(512: the 35.5M-site pack, about 20 minutes)")
    ap.add_argument("--controller-margin-frac", type=float, default=0.25,
                    help="steps run on after settling, as a fraction of the settling time "
                         "(the committed 512^3 comparison used 0.1)")
    ap.add_argument("--pull", choices=list(PULL_FORMATS), default="run",
                    help="pull-table format of the step: 8/16-bit codes with run codes, 8/16-bit codes, "
                         "16-bit codes, or the int32 table")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(sharding the lattice into z-slabs with a halo exchange per step is a design only)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1806_10589_amd import fluxlbm

    cfg = CONFIGS[args.config]
    if cfg.get("batch"):
        return run_batch(args, cfg)
    mask, kw, info = make_workload(cfg)
    print(f"[bench] workload {args.config}: mask {mask.shape}, pore sites {(mask == 0).sum()}",
          file=sys.stderr, flush=True)
    lat = fluxlbm.Lattice(mask, watchdog_every=1000, **kw)
    colour = kw.get("model") == "colour"
    share = pull_share([lat], args.pull)
    if kw.get("model") == "colour":
        z = lat.coords()[:, 2]
        na = (z < cfg["reservoir"]).astype(float)
        lat.init_colour(na, 1.0 - na)
    else:
        lat.init_equilibrium(1.0)
    n = lat.n_sites

    lat.step(args.warmup)
    torch.cuda.synchronize()
    if lat.sync() != fluxlbm.FLBM_OK:
        raise SystemExit("unstable during warm-up")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(lat.stream)
    lat.step(args.steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    status = lat.sync()
    ms_step = ms_total / args.steps
    mlups = n * args.steps / (ms_total * 1e-3) / 1e6
    q_in, q_out, rho_in, _ = lat.boundary()
    print(f"[bench] {args.steps} steps in {ms_total:.1f} ms (wall {wall:.2f} s): {mlups:.1f} MLUPS, "
          f"Q_in {q_in:.6f} Q_out {q_out:.6f} rho_in {rho_in:.6f}", file=sys.stderr, flush=True)

    # per-kernel durations with HIP events on the launch stream
    ms_plane, ms_kernel = lat.profile_kernels(args.profile_steps)
    roofline = roofline_of(args.config, kw, n, share, ms_kernel, ms_plane, args.pull)
    out = {
        "metric": "MLUPS (pore sites) + HBM GB/s; steps-to-flux-tol, learned vs plain",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16dev": "f16-storage/f32"}[kw["precision"]],
        "data": "synthetic",
        "config": {
            "workload": args.config,
            "mask": list(mask.shape),
            "pore_sites": n,
            "inlet_sites": lat.a_in,
            "tau": kw["tau"],
            "q_target": kw["q_target"],
            "precision": kw["precision"],
            "collision": kw.get("model", "bgk"),
            "pull_table": args.pull,
            "tile_share_8bit_16bit": [round(v, 4) for v in share[:2]],
            "run_share_tiles_waves_wide": [round(v, 4) for v in share[2:]],
            **info,
        },
        "hbm_gbs_model": round(mlups * roofline["bytes_per_lup"] / 1e3, 1),
        "status": "ok" if status == fluxlbm.FLBM_OK else "unstable",
        "roofline": roofline,
    }
    lat.close()
    del lat
    torch.cuda.empty_cache()
    if not args.no_copy:
        out["copy_gbs"] = round(copy_bandwidth(torch), 1)
        # the same fractions against the stream copy measured in this run
        out["roofline"]["frac_copy"] = round(roofline["achieved"] / out["copy_gbs"], 4)
        out["roofline"]["frac_survey_copy"] = round(roofline["achieved_survey"] / out["copy_gbs"], 4)
        if roofline.get("traffic_gbs"):
            out["roofline"]["traffic_frac_copy"] = round(roofline["traffic_gbs"] / out["copy_gbs"], 4)
    if args.config == "pack256" and not args.no_pack512:
        out["pack512"] = pack512_line(args)
    if not args.no_controller and args.config == "pack256":
        out["controller_ab"] = controller_ab(args.controller_n, args.controller_margin_frac)
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        out["cpu_baseline"] = cpu_baseline(mask, kw, args.cpu_steps, steps_t1=args.cpu_steps_1_thread)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
