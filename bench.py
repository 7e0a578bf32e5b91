"""Benchmark of the three-phonon linewidth hot path on one MI355X.

A step is one pass of the whole path over the diamond 2-atom cell on a
15x15x15 Gamma-centred mesh (20,250 modes, T = 300 K, adaptive Gaussian
smearing): GPU phonons (FP64) -> linewidths (FP32 projection, FP64 cut and
sums) -> RTA conductivity.  Inputs (force constants, buffers) are resident in
HBM before the timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|fp64]
                    [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3  # TFLOP/s, MI355X vector FP32 and FP32 MFMA (datasheet)

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch) scaled by the copy-kernel calibration
# (fetch x 1.99995, write x 1.0); valid only for the kernel sources hashed
# here, reported as null once they change.
MEASURED_TRAFFIC = {
    "lw_fused": {"sources": ["lw_fused.hip", "lw_common.h", "common.h"],
                 "sha256": "255bd3fdb705aa75efcc7d9c549a4092699d1f8245ea98c12f883dfa4b121677",
                 "bytes": 58784804, "config": "C2"},
}


def fc3_mirror_symmetric(model, rel=1e-12):
    """Phi3(i, j, k) == Phi3(i, k, j) over the COO (duplicates summed)."""
    acc = {}
    for i, j, k, v in zip(model.fc3_i.tolist(), model.fc3_j.tolist(), model.fc3_k.tolist(),
                          model.fc3_val.tolist()):
        acc[(i, j, k)] = acc.get((i, j, k), 0.0) + v
    tol = rel * max(abs(v) for v in acc.values())
    return all(abs(v - acc.get((i, k, j), 0.0)) <= tol for (i, j, k), v in acc.items())


def measured_traffic(kernel, config):
    import hashlib
    rec = MEASURED_TRAFFIC.get(kernel)
    if rec is None or rec["config"] != config:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, "paper_2602_23728_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return rec["bytes"] if h.hexdigest() == rec["sha256"] else None
METRIC = "3-phonon linewidths: modes/s and MFMA util; speedup of split/surrogate at κ tol"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-q", type=int, default=200)
    ap.add_argument("--form", default="plain", choices=["plain", "learned"],
                    help="learned: the learned form against plain FP32 (full mesh and wedge)")
    ap.add_argument("--train-steps", type=int, default=200)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


def profile_read(K):
    rec = (K.KernelTime * 64)()
    n = ctypes.c_int32()
    K._check(K.lib().kaldo_profile_end(rec, 64, ctypes.byref(n)))
    return {rec[i].name.decode(): (int(rec[i].launches), float(rec[i].total_ms))
            for i in range(min(n.value, 64))}


def cpu_baseline(cfg, model, nq_sample, seed=0):
    """The oracle as it stands, on a bounded sample of the same workload."""
    from oracle import linewidths as olw
    from oracle import phonons as oph
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = 1
    t0 = time.perf_counter()
    om, ev, ve = oph.phonons(model, cfg.mesh)
    t_ph = time.perf_counter() - t0
    nq = om.shape[0]
    qs = sorted(np.random.default_rng(seed).choice(nq, nq_sample, replace=False).tolist())
    stats = {}
    t0 = time.perf_counter()
    olw.crystal_linewidths(model, cfg.mesh, om, ev, ve, cfg.temperature, cfg.broadening,
                           q_list=qs, stats=stats)
    t_lw = time.perf_counter() - t0
    est = t_ph + t_lw * nq / nq_sample
    n_modes = nq * 3 * model.n_basis
    return dict(value=n_modes / est, unit="modes/s", cores=int(threads), kind="oracle",
                sample=(f"oracle phonons on all {nq} q-points ({t_ph:.1f} s) + linewidths on "
                        f"{nq_sample} seeded q-points ({nq_sample * 3 * model.n_basis} modes, "
                        f"{t_lw:.1f} s), extrapolated linearly to {nq} q-points"),
                est_total_s=est), stats


def bench_gamma_point(a, cfg, model, c, prec, K, torch):
    """Gamma-point solid: host FP64 eigenproblem once (setup), then the GPU
    linewidth pass timed."""
    t0 = time.perf_counter()
    om_h, E_h = K.phonons_gamma(model.n_basis, model.mass, model.fc2)
    t_eig = time.perf_counter() - t0
    om = torch.as_tensor(om_h).cuda()
    E = torch.as_tensor(E_h).cuda()
    n = len(om_h)
    ws = torch.empty(int(K.lib().kaldo_linewidths_gamma_workspace(c.handle, prec)),
                     dtype=torch.uint8, device="cuda")
    gam = torch.empty(n, dtype=torch.float64, device="cuda")

    def step():
        K.linewidths_gamma(c, om, E, cfg.temperature, cfg.broadening, prec, workspace=ws, out=gam)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    K.lib().kaldo_profile_begin()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = profile_read(K)
    ms = 1e3 * elapsed / a.steps
    print(f"bench: {ms:.3f} ms/step; kernels: " +
          ", ".join(f"{k} {v[1] / v[0]:.3f} ms x{v[0] // a.steps}" for k, v in prof.items()),
          file=sys.stderr, flush=True)
    # Executed work of the vertex GEMM: 2 * 128^2 * n_pad FLOP per live tile,
    # a tile (I <= J) of mode mu being live when the physical frequency ranges
    # of blocks I and J can meet the 2-sigma cut in either order.
    npad = (n + 127) // 128 * 128
    nt = npad // 128
    phys = om_h / (2 * np.pi) >= cfg.broadening.nu_min_thz
    lo = np.full(nt, np.inf)
    hi = np.full(nt, -np.inf)
    for I in range(nt):
        sel = np.arange(I * 128, min(n, I * 128 + 128))
        sel = sel[phys[sel]]
        if len(sel):
            lo[I], hi[I] = om_h[sel].min(), om_h[sel].max()
    reach = 2 * (2 * np.pi * cfg.broadening.sigma_thz) * (1 + 1e-12) + 1e-9
    w = om_h[phys][:, None, None]
    l1, h1, l2, h2 = lo[None, :, None], hi[None, :, None], lo[None, None, :], hi[None, None, :]
    def can(l1, h1, l2, h2):
        return (((w + l1 - h2) < reach) & ((w + h1 - l2) > -reach)) | \
               (((w - h1 - h2) < reach) & ((w - l1 - l2) > -reach))
    I, J = np.meshgrid(np.arange(nt), np.arange(nt), indexing="ij")
    valid = (I <= J)[None] & (lo[:, None] <= hi[:, None])[None] & (lo[None, :] <= hi[None, :])[None]
    live = valid & (can(l1, h1, l2, h2) | ((I != J)[None] & can(l2, h2, l1, h1)))
    flop = float(live.sum()) * 2.0 * 128 * 128 * npad
    gemm_ms = sum(v[1] for k, v in prof.items() if k.startswith("gm_gemm")) / a.steps
    split = a.precision == "bf16x3"
    achieved = (3.0 if split else 1.0) * flop / (gemm_ms * 1e-3) / 1e12
    peak = 2500.0 if split else FP32_VECTOR_PEAK
    roof = dict(bound="mfma", achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
                traffic=None, kernel="gm_gemm", kernel_ms_per_step=gemm_ms,
                work_model="live tiles" + (" (three bf16 products counted)" if split else ""),
                live_tiles=int(live.sum()), dense_tiles=int(phys.sum()) * nt * (nt + 1) // 2)
    print(json.dumps({"metric": METRIC, "value": n / (ms * 1e-3), "unit": "modes/s",
                      "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "bf16x3" if split else "f32", "data": "synthetic",
                      "config": {"workload": f"{cfg.name}: {cfg.description}", "modes": n,
                                 "precision": a.precision},
                      "roofline": roof,
                      "host_eigensolver_s": t_eig,
                      "kernels_ms_per_step": {k: v[1] / a.steps for k, v in prof.items()}}))


def bench_learned(a, cfg, model, c, K, torch):
    """The learned form on a crystal mesh, against the plain FP32 path on every
    mode (the conductivity reference) and on the irreducible wedge.  Each of
    the three chains (phonons -> linewidths -> conductivity) is timed over
    `steps` repetitions; the wedge itself is host set-up."""
    from paper_2602_23728_amd import learned as L
    from synthetic import draws as D
    mesh, T, b = cfg.mesh, cfg.temperature, cfg.broadening
    nq = int(np.prod(mesh))
    nb3 = c.nb3
    wedge = L.Wedge(model.lattice, model.frac, model.mass, mesh)
    kap = torch.empty(3, 3, dtype=torch.float64, device="cuda")
    state = {}

    def full():
        om, ev, ve = K.phonons(c, mesh)
        g = K.linewidths(c, mesh, om, ev, ve, T, b, K.FP32)
        K.kappa_rta(c, mesh, om, ve, g, T, b.nu_min_thz, out=kap)
        return kap.clone()

    def ibz():
        om, ev, ve = K.phonons(c, mesh)
        g = L.plain_ibz_linewidths(c, wedge, om, ev, ve, T, b, K.FP32)
        K.kappa_rta(c, mesh, om, ve, g, T, b.nu_min_thz, out=kap)
        return kap.clone()

    def learned():
        om, ev, ve = K.phonons(c, mesh)
        cand = L.candidate_modes(wedge, om, nb3, b.nu_min_thz)
        if "draws" not in state or len(state["cand"]) != len(cand):
            state["cand"] = cand
            state["draws"] = D.surrogate_draws(len(cand), K.surrogate_feature_count(c), members=5,
                                               seed=0)
        res = L.learned_linewidths(c, wedge, om, ev, ve, T, b, cand, state["draws"],
                                   steps=a.train_steps, lr=2e-2, tol=0.01)
        K.kappa_rta(c, mesh, om, ve, res.gamma, T, b.nu_min_thz, out=kap)
        state["res"] = res
        return kap.clone()

    def timed(fn, name):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        K.lib().kaldo_profile_begin()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            k = fn()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / a.steps
        prof = profile_read(K)
        print(f"bench[{name}]: {ms:.3f} ms/step; kernels: " +
              ", ".join(f"{kk} {v[1] / a.steps:.3f} ms" for kk, v in prof.items()),
              file=sys.stderr, flush=True)
        return ms, k.cpu().numpy(), {kk: v[1] / a.steps for kk, v in prof.items()}

    ms_full, k_full, p_full = timed(full, "plain-full")
    ms_ibz, k_ibz, p_ibz = timed(ibz, "plain-wedge")
    ms_lrn, k_lrn, p_lrn = timed(learned, "learned")
    res = state["res"]

    def rel(k):
        kbar = np.trace(k_full) / 3
        return float(max(abs(np.trace(k) / 3 - kbar) / kbar, np.max(np.abs(k - k_full)) / kbar))

    n_modes = nq * nb3
    n_rest = len(state["cand"]) - res.n_train - res.n_held
    print(json.dumps({
        "metric": METRIC, "value": n_modes / (ms_lrn * 1e-3), "unit": "modes/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_lrn, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.description}", "modes": n_modes,
                   "mesh": list(mesh), "form": "learned"},
        "plain_full_ms": ms_full, "plain_wedge_ms": ms_ibz,
        "speedup_vs_plain_full": ms_full / ms_lrn, "speedup_vs_plain_wedge": ms_ibz / ms_lrn,
        "kappa_rel_err_learned": rel(k_lrn), "kappa_rel_err_wedge": rel(k_ibz),
        "kappa_trace_over_3": float(np.trace(k_full) / 3),
        "irreducible_q": int(wedge.n_ir), "candidates": int(len(state["cand"])),
        "train": res.n_train, "held_out": res.n_held, "fallback": res.n_fallback,
        "fallback_frac_of_rest": res.n_fallback / max(1, n_rest), "tau": res.tau,
        "train_steps": a.train_steps,
        "kernels_ms_per_step": {"plain_full": p_full, "plain_wedge": p_ibz, "learned": p_lrn},
    }))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: kaldo runs on one GPU (asked for --gpus {a.gpus}); sharding the "
              "path over several GPUs is described in the design notes, not implemented.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if a.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": x.numel() * 4,
                          "copy_calibration_bytes_written": y.numel() * 4, "launches": 3}))
        return

    from paper_2602_23728_amd import kaldo as K
    from synthetic import configs

    cfg = configs.CONFIGS[a.config]
    model = configs.model_for(cfg)
    prec = {"fp32": K.FP32, "fp64": K.FP64, "bf16x3": K.BF16X3}[a.precision]
    torch.cuda.set_device(0)
    c = K.Crystal.from_model(model)
    if cfg.mesh == (1, 1, 1):
        return bench_gamma_point(a, cfg, model, c, prec, K, torch)
    if a.form == "learned":
        return bench_learned(a, cfg, model, c, K, torch)
    mesh = cfg.mesh
    nq = int(np.prod(mesh))
    nb3 = c.nb3
    n_modes = nq * nb3
    dev = torch.device("cuda")
    om = torch.empty(nq, nb3, dtype=torch.float64, device=dev)
    ev = torch.empty(nq, nb3, nb3, 2, dtype=torch.float64, device=dev)
    ve = torch.empty(nq, nb3, 3, dtype=torch.float64, device=dev)
    gam = torch.empty(nq, nb3, dtype=torch.float64, device=dev)
    kap = torch.empty(3, 3, dtype=torch.float64, device=dev)
    ws = torch.empty(K.linewidths_workspace(c, mesh, prec), dtype=torch.uint8, device=dev)

    def step():
        K.phonons(c, mesh, out=(om, ev, ve))
        K.linewidths(c, mesh, om, ev, ve, cfg.temperature, cfg.broadening, prec,
                     workspace=ws, out=gam)
        K.kappa_rta(c, mesh, om, ve, gam, cfg.temperature, cfg.broadening.nu_min_thz, out=kap)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    print(f"bench: warmup done ({a.warmup} steps), timing {a.steps} steps", file=sys.stderr,
          flush=True)
    K.lib().kaldo_profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = profile_read(K)
    ms_per_step = 1e3 * elapsed / a.steps
    kappa = kap.cpu().numpy()
    print(f"bench: {ms_per_step:.3f} ms/step; kernels: " +
          ", ".join(f"{k} {v[1] / v[0]:.3f} ms" for k, v in prof.items()), file=sys.stderr,
          flush=True)

    dom, (launches, total) = max(prof.items(), key=lambda kv: kv[1][1])
    avg_ms = total / launches

    base, stats = (None, {})
    if not a.no_cpu_baseline:
        base, stats = cpu_baseline(cfg, model, a.cpu_sample_q)
        print(f"bench: cpu baseline {base['value']:.1f} modes/s", file=sys.stderr, flush=True)
    # Work model per mode: dense-block F_blk = 8 N_q (n_p + 2 nb3^3) and the
    # pruned F_pr = 8 N_q (f_blk n_p + f_pass nb3^4) with the oracle-measured
    # fractions of partner blocks / candidates that pass the 2-sigma cut.
    from collections import Counter
    n_p = len(Counter(zip(model.fc3_j.tolist(), model.fc3_k.tolist())))
    F_blk = 8.0 * nq * (n_p + 2 * nb3 ** 3)
    roof = None
    if dom in ("lw_crystal", "lw_fused") and stats:
        f_blk = stats["blocks_pass"] / max(1, stats["blocks"])
        f_pass = stats["passed"] / max(1, stats["cand"])
        F_pr = 8.0 * nq * (f_blk * n_p + f_pass * nb3 ** 4)
        achieved = F_pr * n_modes / (avg_ms * 1e-3) / 1e12
        # With Phi3 symmetric in its last two slots the fused kernel visits each
        # mirrored partner pair (q1, q2) once: on average (N_q + 1) / 2 partner
        # points per q (one q1 == q2 point per q on average), so it executes
        # about half of the ordered-pair work F_pr counts.
        f_exec = (nq + 1) / (2.0 * nq) if (dom == "lw_fused" and fc3_mirror_symmetric(model)) else 1.0
        roof = dict(bound="alu", achieved=achieved, peak=FP32_VECTOR_PEAK, unit="TFLOP/s",
                    frac=achieved / FP32_VECTOR_PEAK, traffic=measured_traffic(dom, cfg.name),
                    kernel=dom, kernel_ms=avg_ms, work_model="pruned, ordered partner pairs",
                    flop_per_mode=F_pr, f_blk=f_blk, f_pass=f_pass,
                    executed_fraction=f_exec, executed_tflops=achieved * f_exec,
                    executed_frac=achieved * f_exec / FP32_VECTOR_PEAK,
                    dense_equiv_tflops=F_blk * n_modes / (avg_ms * 1e-3) / 1e12)
    if dom.startswith("lw_mfma"):
        # Dense MFMA kernel: per (q, swept partner q1, live branch s) two complex
        # 16x16x16 products (T = B_s eta2, V = eta1^T T), each two real 16x16x32
        # products, i.e. 65,536 FLOP; the BF16x3 form issues three BF16 products
        # per real product.  Partners: (N_q + 1) / 2 per q on average when the
        # mirrored pair is visited once, else N_q.
        om_h = om.cpu().numpy()
        n_live = int(np.sum(om_h / (2 * np.pi) >= cfg.broadening.nu_min_thz))
        partners = (nq + 1) / 2.0 if fc3_mirror_symmetric(model) else float(nq)
        split = prec == K.BF16X3
        flop = n_live * partners * 65536.0 * (3 if split else 1)
        achieved = flop / (avg_ms * 1e-3) / 1e12
        peak = 2500.0 if split else FP32_VECTOR_PEAK
        roof = dict(bound="mfma", achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
                    traffic=None, kernel=dom, kernel_ms=avg_ms,
                    work_model="dense 16x16 tiles per (q, partner, live branch)"
                               + (", three BF16 products counted" if split else ""),
                    flop_per_launch=flop)
    out = {
        "metric": METRIC,
        "value": n_modes / (ms_per_step * 1e-3),
        "unit": "modes/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {K.FP32: "f32", K.FP64: "f64", K.BF16X3: "bf16x3"}[prec],
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.description}", "modes": n_modes,
                   "mesh": list(mesh), "precision": a.precision},
        "roofline": roof,
        "cpu_baseline": base,
        "kernels_ms": {k: v[1] / v[0] for k, v in prof.items()},
        "kappa_trace_over_3": float(np.trace(kappa) / 3),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
