"""Benchmark of the three-phonon linewidth hot path on one MI355X.

A step is one pass of the whole path over the diamond 2-atom cell on a
24x24x24 Gamma-centred mesh (82,944 modes, the largest configuration; T =
300 K, adaptive Gaussian smearing): GPU phonons (FP64) -> linewidths (FP64
projection, FP64 cut, weights and sums: the paper's arithmetic) -> RTA
conductivity.  Inputs (force constants, buffers) are resident in HBM before
the timed region.  Prints one JSON line.

Beside the headline the line carries, each timed on the GPU the same way:
  fp32        the same step with the FP32 projection, and its speedup;
  c3_split    the perovskite 12^3 mesh in FP32 and in BF16x3 (split
              precision on the matrix cores): step times, speedup, and the
              conductivity difference between the two forms;
  c4          the 512-atom Gamma-point glass: FP32 and BF16x3 projection
              times and their fraction of the FP32 / BF16 matrix-core peak,
              for the vertex GEMM alone and for the whole projection;
  bte_c2      the full BTE on the diamond 15^3 mesh (scattering matrix and
              its direct inversion);
  qhgk        QHGK conductivity of the 512-atom glass (FP64 matrix cores) and
              the interband term of the perovskite 12^3 mesh;
  isotope     isotope scattering of every mode of the headline mesh with
              natural silicon, and the conductivity with it added;
  wedge       the irreducible wedge (representatives' modes + star map)
              against the full mesh on the diamond 15^3 (FP64) and perovskite
              12^3 (FP32) meshes;
  tsweep      Gamma at 16 temperatures from the temperature cache of the
              headline mesh (and of its irreducible wedge), against the
              direct path per temperature.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C5]
                    [--precision fp64|fp32|bf16x3] [--no-cpu-baseline]
                    [--no-extras] [--form plain|learned|bte|tsweep|isotope|qhgk] [--copy-calibration]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X datasheet peaks, TFLOP/s (dense).
FP32_PEAK = 157.3   # FP32 vector = FP32 matrix core
FP64_PEAK = 78.6    # FP64 vector = FP64 matrix core
BF16_PEAK = 2500.0  # BF16 matrix core

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch) scaled by the copy-kernel calibration; valid
# only for the kernel sources hashed here, reported as null once they change.
MEASURED_TRAFFIC = {
    ("lw_fused", "C2", "fp32"): {"sources": ["lw_fused.hip", "lw_common.h", "common.h"],
                                 "sha256": "7173bbcd813ced92d4a22b9bce87910d247d01854ef917948045030fd2e64b0c",
                                 "bytes": 29167602},
    ("lw_fused", "C5", "fp64"): {"sources": ["lw_fused.hip", "lw_common.h", "common.h"],
                                 "sha256": "7173bbcd813ced92d4a22b9bce87910d247d01854ef917948045030fd2e64b0c",
                                 "bytes": 20506261099},
    ("tc_gamma", "C5", "fp64"): {"sources": ["tcache.hip", "lw_common.h", "common.h"],
                                 "sha256": "eac6a619af40cad7b795df420a1461fb42233db14a29bebc24f55a8630e74f5b",
                                 "bytes": 2471809537},
}


def fc3_mirror_symmetric(model, rel=1e-12):
    """Phi3(i, j, k) == Phi3(i, k, j) over the COO (duplicates summed)."""
    acc = {}
    for i, j, k, v in zip(model.fc3_i.tolist(), model.fc3_j.tolist(), model.fc3_k.tolist(),
                          model.fc3_val.tolist()):
        acc[(i, j, k)] = acc.get((i, j, k), 0.0) + v
    tol = rel * max(abs(v) for v in acc.values())
    return all(abs(v - acc.get((i, k, j), 0.0)) <= tol for (i, j, k), v in acc.items())


def measured_traffic(kernel, config, precision="fp32"):
    import hashlib
    rec = MEASURED_TRAFFIC.get((kernel, config, precision))
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, "paper_2602_23728_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return rec["bytes"] if h.hexdigest() == rec["sha256"] else None


METRIC = "3-phonon linewidths: modes/s and MFMA util; speedup of split/surrogate at κ tol"


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C5")
    ap.add_argument("--precision", default="fp64", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU time the oracle sample may take (the sample grows in q-point "
                         "batches until it does)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline step (no FP32, C3 split or C4 legs)")
    ap.add_argument("--form", default="plain", choices=["plain", "learned", "bte", "tsweep", "isotope", "qhgk"],
                    help="learned: the learned form against plain FP32 (full mesh and wedge); "
                         "bte: only the full-BTE leg (diamond 15^3); tsweep: only the "
                         "temperature-sweep leg on --config; isotope: only the isotope leg; qhgk: only "
                         "the QHGK leg")
    ap.add_argument("--train-steps", type=int, default=200)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args(argv)


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def profile_read(K):
    rec = (K.KernelTime * 64)()
    n = ctypes.c_int32()
    K._check(K.lib().kaldo_profile_end(rec, 64, ctypes.byref(n)))
    return {rec[i].name.decode(): (int(rec[i].launches), float(rec[i].total_ms))
            for i in range(min(n.value, 64))}


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(cfg, model, seconds, seed=0):
    """The oracle as it stands, on a bounded sample of the same workload: its
    phonons on every q-point, then its linewidths on seeded q-points taken in
    batches of 8 until `seconds` have passed, extrapolated linearly to the
    mesh.  Also returns the oracle's pass counts on that sample (the pruned
    work model)."""
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
    order = np.random.default_rng(seed).permutation(nq).tolist()
    stats_all = {}
    done = 0
    t0 = time.perf_counter()
    while done < nq and (done < 8 or time.perf_counter() - t0 < seconds):
        qs = sorted(order[done:done + 8])
        st = {}
        olw.crystal_linewidths(model, cfg.mesh, om, ev, ve, cfg.temperature, cfg.broadening,
                               q_list=qs, stats=st)
        for k, v in st.items():
            stats_all[k] = stats_all.get(k, 0) + v
        done += len(qs)
    t_lw = time.perf_counter() - t0
    est = t_ph + t_lw * nq / done
    n_modes = nq * 3 * model.n_basis
    cpu_model, nproc = host_info()
    return dict(value=n_modes / est, unit="modes/s", cores=int(threads), kind="oracle",
                nproc=nproc, cpu_model=cpu_model,
                sample=(f"oracle phonons on all {nq} q-points ({t_ph:.1f} s) + linewidths on "
                        f"{done} seeded q-points ({done * 3 * model.n_basis} modes, "
                        f"{t_lw:.1f} s), extrapolated linearly to {nq} q-points"),
                est_total_s=est), stats_all, om


def pruned_work(model, nq, stats, om_oracle, nu_min):
    """Pruned work model of the crystal projection (method's own minimum under
    the 2-sigma cut), from the oracle's pass counts on its sample: per
    physical mode F_pr = 8 N_q (f_blk n_p + f_pass (3N_b)^4) FLOP, f_blk the
    share of (mode, q1) blocks with a pair passing in either process and
    f_pass the share of (mode, q1, s', s'') candidates passing in either
    process, both over physical modes.  Total = F_pr x physical modes."""
    from collections import Counter
    nb3 = 3 * model.n_basis
    n_p = len(Counter(zip(model.fc3_j.tolist(), model.fc3_k.tolist())))
    f_blk = stats["mode_blocks_pass"] / (stats["mode_phys"] * nq)
    f_pass = stats["mode_pass"] / (stats["mode_phys"] * nq * nb3 * nb3)
    F_pr = 8.0 * nq * (f_blk * n_p + f_pass * nb3 ** 4)
    n_phys = int(np.sum(om_oracle / (2 * np.pi) >= nu_min))
    F_blk = 8.0 * nq * (n_p + 2 * nb3 ** 3)
    return dict(f_blk=f_blk, f_pass=f_pass, flop_per_mode=F_pr, n_p=n_p,
                physical_modes=n_phys, total_flop=F_pr * n_phys, dense_flop_per_mode=F_blk)


def crystal_step(K, torch, c, cfg, prec):
    """Buffers and the step closure for one crystal config and precision."""
    mesh = cfg.mesh
    nq = int(np.prod(mesh))
    nb3 = c.nb3
    dev = torch.device("cuda")
    om = torch.empty(nq, nb3, dtype=torch.float64, device=dev)
    ev = torch.empty(nq, nb3, nb3, 2, dtype=torch.float64, device=dev)
    ve = torch.empty(nq, nb3, 3, dtype=torch.float64, device=dev)
    gam = torch.empty(nq, nb3, dtype=torch.float64, device=dev)
    kap = torch.empty(3, 3, dtype=torch.float64, device=dev)
    ws = torch.empty(max(1, K.linewidths_workspace(c, mesh, prec)), dtype=torch.uint8, device=dev)

    def step():
        K.phonons(c, mesh, out=(om, ev, ve))
        K.linewidths(c, mesh, om, ev, ve, cfg.temperature, cfg.broadening, prec,
                     workspace=ws, out=gam)
        K.kappa_rta(c, mesh, om, ve, gam, cfg.temperature, cfg.broadening.nu_min_thz, out=kap)

    return step, dict(om=om, ev=ev, ve=ve, gam=gam, kap=kap)


def timed(K, torch, step, steps, warmup, name, plain=False):
    """Wall time per step over `steps` steps after `warmup`, and the library's
    per-kernel HIP-event times.  By default the kernels are timed in the same
    steps (the headline: its roofline divides by the kernel's average over the
    timed region).  With plain=True the steps are timed without the
    per-kernel events (two event records per launch cost several microseconds
    of GPU time each, which matters for the launch-heavy legs) and the kernel
    times come from a second pass of as many steps."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    log(f"{name}: warmup done ({warmup} steps), timing {steps} steps")

    def run():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    if plain:
        elapsed = run()
        K.lib().kaldo_profile_begin()
        run()
    else:
        K.lib().kaldo_profile_begin()
        elapsed = run()
    prof = profile_read(K)
    ms = 1e3 * elapsed / steps
    log(f"{name}: {ms:.3f} ms/step{' (kernels from a profiled pass)' if plain else ''}; kernels: " +
        ", ".join(f"{k} {v[1] / v[0]:.3f} ms" for k, v in prof.items()))
    return ms, prof


def gamma_point_live_flop(om_h, broadening, sym=True):
    """Executed work of the vertex GEMM: 2 * 128^2 * n_pad FLOP per live tile,
    a tile (I <= J for a symmetric Phi3) of mode mu being live when the
    physical frequency ranges of blocks I and J can meet the 2-sigma cut (in
    either order of the pair)."""
    n = len(om_h)
    npad = (n + 127) // 128 * 128
    nt = npad // 128
    phys = om_h / (2 * np.pi) >= broadening.nu_min_thz
    lo = np.full(nt, np.inf)
    hi = np.full(nt, -np.inf)
    for I in range(nt):
        sel = np.arange(I * 128, min(n, I * 128 + 128))
        sel = sel[phys[sel]]
        if len(sel):
            lo[I], hi[I] = om_h[sel].min(), om_h[sel].max()
    reach = 2 * (2 * np.pi * broadening.sigma_thz) * (1 + 1e-12) + 1e-9
    w = om_h[phys][:, None, None]
    l1, h1, l2, h2 = lo[None, :, None], hi[None, :, None], lo[None, None, :], hi[None, None, :]

    def can(l1, h1, l2, h2):
        return (((w + l1 - h2) < reach) & ((w + h1 - l2) > -reach)) | \
               (((w - h1 - h2) < reach) & ((w - l1 - l2) > -reach))
    I, J = np.meshgrid(np.arange(nt), np.arange(nt), indexing="ij")
    ok = (lo[:, None] <= hi[:, None])[None] & (lo[None, :] <= hi[None, :])[None]
    if sym:
        live = (I <= J)[None] & ok & (can(l1, h1, l2, h2) | ((I != J)[None] & can(l2, h2, l1, h1)))
    else:
        live = ok & can(l1, h1, l2, h2)
    return float(live.sum()) * 2.0 * 128 * 128 * npad, int(live.sum()), int(phys.sum())


def gamma_point_leg(a, K, torch, cfg, model, steps, warmup):
    """Gamma-point glass: host FP64 eigenproblem once (set-up), then FP32 and
    BF16x3 projections timed; fractions of the matrix-core peak for the
    vertex GEMM alone and for the whole projection (A values + SpMM + GEMM)."""
    c = K.Crystal.from_model(model)
    t0 = time.perf_counter()
    om_h, E_h = K.phonons_gamma(model.n_basis, model.mass, model.fc2)
    t_eig = time.perf_counter() - t0
    om = torch.as_tensor(om_h).cuda()
    E = torch.as_tensor(E_h).cuda()
    n = len(om_h)
    flop, live, n_phys = gamma_point_live_flop(om_h, cfg.broadening, fc3_mirror_symmetric(model))
    out = dict(modes=n, host_eigensolver_s=t_eig, live_tiles=live)
    for name, prec in (("fp32", K.FP32), ("bf16x3", K.BF16X3)):
        ws = torch.empty(int(K.lib().kaldo_linewidths_gamma_workspace(c.handle, prec)),
                         dtype=torch.uint8, device="cuda")
        gam = torch.empty(n, dtype=torch.float64, device="cuda")

        def step():
            K.linewidths_gamma(c, om, E, cfg.temperature, cfg.broadening, prec, workspace=ws,
                               out=gam)
        ms, prof = timed(K, torch, step, steps, warmup, f"{cfg.name} {name}", plain=True)
        per = {k: v[1] / steps for k, v in prof.items()}
        gemm = sum(v for k, v in per.items() if k.startswith("gm_gemm"))
        proj = gemm + sum(v for k, v in per.items() if k in ("gm_avals", "gm_spmm", "gm_fused"))
        split = prec == K.BF16X3
        f = (3.0 if split else 1.0) * flop
        peak = BF16_PEAK if split else FP32_PEAK
        out[name] = dict(ms_per_step=ms, modes_per_s=n / (ms * 1e-3), gemm_ms=gemm,
                         projection_ms=proj,
                         gemm_tflops=f / (gemm * 1e-3) / 1e12,
                         gemm_frac=f / (gemm * 1e-3) / 1e12 / peak,
                         projection_frac=f / (proj * 1e-3) / 1e12 / peak, peak=peak,
                         kernels_ms_per_step=per)
        del ws
    out["split_speedup"] = out["fp32"]["ms_per_step"] / out["bf16x3"]["ms_per_step"]
    c.close()
    return out


def bte_leg(K, torch, steps, warmup):
    """Full BTE on the diamond 15^3 mesh (20,250 modes): the dense FP64
    scattering matrix (3.3 GB) and its direct inversion (Eq. inverse) by the
    blocked LU, timed per step (the factorisation overwrites the matrix, so
    every step rebuilds it); the LU runs on the coupled modes (the decoupled
    ones have lambda = 0), its trailing updates on the FP64 matrix cores,
    (2/3) n_c^3 FLOP in all."""
    from synthetic import configs
    cfg = configs.CONFIGS["C2"]
    model = configs.model_for(cfg)
    c = K.Crystal.from_model(model)
    mesh = cfg.mesh
    nq = int(np.prod(mesh))
    n = nq * c.nb3
    om, ev, ve = K.phonons(c, mesh)
    ws = torch.empty(K.bte_workspace(c, mesh), dtype=torch.uint8, device="cuda")
    mat = torch.empty(n, n, dtype=torch.float64, device="cuda")
    g0 = torch.empty(n, dtype=torch.float64, device="cuda")
    state = {}

    def step():
        K.scattering_matrix(c, mesh, om, ev, ve, cfg.temperature, cfg.broadening, workspace=ws,
                            out=(mat, g0))
        state["lk"] = K.bte_solve(c, mesh, om, ve, g0, cfg.temperature,
                                  cfg.broadening.nu_min_thz, mat, workspace=ws)

    ms, prof = timed(K, torch, step, steps, warmup, "C2 full BTE", plain=True)
    c.device_status()
    per = {k: v[1] / steps for k, v in prof.items()}
    solve_side = ("bte_compact_index", "bte_compact_cols", "bte_gather3", "bte_scatter3",
                  "bte_copy3", "bte_kappa")
    build = sum(v for k, v in per.items() if k.startswith("bte_") and k not in solve_side)
    lu = sum(v for k, v in per.items() if k.startswith("lu_"))
    upd = per.get("lu_update", 0.0)
    # the factorisation runs on the coupled modes only (nu >= nu_min and
    # Gamma0 above 1e-8 of its largest value)
    om_h, g0_h = om.cpu().numpy().ravel(), g0.cpu().numpy()
    coupled = int(np.sum((om_h / (2 * np.pi) >= cfg.broadening.nu_min_thz) &
                         (g0_h > 1e-8 * g0_h.max()) & (g0_h > 0)))
    flop_lu = 2.0 / 3.0 * float(coupled) ** 3
    kap = state["lk"][1].cpu().numpy()
    out = dict(modes=n, coupled_modes=coupled, matrix_bytes=n * n * 8, ms_per_step=ms,
               build_ms=build, lu_solve_ms=lu,
               lu_update_ms=upd, lu_tflops=flop_lu / (lu * 1e-3) / 1e12,
               lu_frac_fp64=flop_lu / (lu * 1e-3) / 1e12 / FP64_PEAK,
               kappa_inv_trace_over_3=float(np.trace(kap) / 3), kernels_ms_per_step=per)
    del mat, ws
    c.close()
    return out


def tsweep_leg(K, torch, cfg, model, c, steps, warmup, n_temps=16, direct_gamma=None):
    """Temperature sweep from the cache (multi-temperature optimisation):
    the FP64 cache of the full mesh built once (count + record passes, timed
    as set-up), then Gamma at n_temps temperatures per step (two batches of
    8, one pass over the entries each), and the same for the irreducible
    wedge (cache of the representatives' modes, star-mapped per T).
    Roofline of tc_gamma: algorithmic HBM bytes per launch = 24 per entry
    (8-byte partner pair + 16-byte factors) + 8 (N + 1) row pointers + 8 NT N
    outputs + 8 NT N populations read once, N modes, NT = 8."""
    from paper_2602_23728_amd import learned as L
    mesh = cfg.mesh
    nq = int(np.prod(mesh))
    n_modes = nq * c.nb3
    om, ev, ve = K.phonons(c, mesh)
    b = cfg.broadening
    temps = np.linspace(100.0, 1600.0, n_temps)
    ws = torch.empty(K.tcache_workspace(c, mesh, K.FP64), dtype=torch.uint8, device="cuda")
    t0 = time.perf_counter()
    K.lib().kaldo_profile_begin()
    cache = K.tcache_build(c, mesh, om, ev, ve, b, K.FP64, workspace=ws)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    bprof = profile_read(K)
    c.device_status()
    log(f"{cfg.name} tcache: {cache.n_entries} entries ({cache.nbytes / 1e9:.2f} GB), "
        f"build {build_s * 1e3:.1f} ms")
    gws = torch.empty(K.tcache_gamma_workspace(c, mesh), dtype=torch.uint8, device="cuda")
    out = torch.empty(n_temps, nq, c.nb3, dtype=torch.float64, device="cuda")

    def step():
        K.tcache_gamma(c, cache, om, b.nu_min_thz, temps, workspace=gws, out=out)
    ms, prof = timed(K, torch, step, steps, warmup, f"{cfg.name} sweep of {n_temps} T", plain=True)
    c.device_status()
    launches, total = prof["tc_gamma"]
    avg = total / launches
    nt = 8
    alg = 24.0 * cache.n_entries + 8.0 * (n_modes + 1) + 2 * 8.0 * nt * n_modes
    res = dict(temperatures=n_temps, entries=cache.n_entries, cache_bytes=cache.nbytes,
               build_ms=build_s * 1e3,
               build_kernels_ms={k: v[1] for k, v in bprof.items()},
               ms_per_step=ms, ms_per_temperature=ms / n_temps,
               modes_temperatures_per_s=n_modes * n_temps / (ms * 1e-3),
               tc_gamma_ms=avg,
               roofline=dict(bound="hbm", achieved=alg / (avg * 1e-3) / 1e9, peak=8000.0,
                             unit="GB/s", frac=alg / (avg * 1e-3) / 1e9 / 8000.0,
                             traffic=measured_traffic("tc_gamma", cfg.name, "fp64"),
                             kernel="tc_gamma", algorithmic_bytes=alg),
               kernels_ms_per_step={k: v[1] / steps for k, v in prof.items()})
    if direct_gamma is not None:
        # the sweep at 300 K against the direct FP64 linewidths of the headline
        g300 = K.tcache_gamma(c, cache, om, b.nu_min_thz, [cfg.temperature])[0]
        d = direct_gamma
        sel = d > 1e-3 * d.max()
        res["max_rel_diff_vs_direct_300K"] = float(((g300 - d).abs()[sel] / d[sel]).max())
    del cache, out
    # the wedge: representatives only, star-mapped at every temperature
    w = L.Wedge(model.lattice, model.frac, model.mass, mesh)
    sub = torch.from_numpy(w.rep_modes(c.nb3)).cuda()
    t0 = time.perf_counter()
    wc = K.tcache_build(c, mesh, om, ev, ve, b, K.FP64, subset=sub, workspace=ws)
    torch.cuda.synchronize()
    wbuild = time.perf_counter() - t0
    g_ir = torch.empty(n_temps, nq, c.nb3, dtype=torch.float64, device="cuda")
    g_full = torch.empty_like(g_ir)

    def wstep():
        K.tcache_gamma(c, wc, om, b.nu_min_thz, temps, workspace=gws, out=g_ir)
        for k in range(n_temps):
            K.star_map(mesh, c.nb3, w.ir_dev, om, g_ir[k], out=g_full[k])
    wms, _ = timed(K, torch, wstep, steps, warmup, f"{cfg.name} wedge sweep of {n_temps} T", plain=True)
    c.device_status()
    res["wedge"] = dict(irreducible_q=int(w.n_ir), entries=wc.n_entries, build_ms=wbuild * 1e3,
                        ms_per_step=wms, ms_per_temperature=wms / n_temps)
    return res


def peaks_leg(torch):
    """Rates re-measured on this device, beside the datasheet peaks the
    roofline objects use: a 1 GiB device-to-device copy (HBM read + write
    bytes per second) and plain library matrix products (torch.matmul on
    contiguous square operands) in FP64, FP32 and BF16."""
    out = {}
    x = torch.empty(256 << 20, dtype=torch.float32, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    out["hbm_copy_GBps"] = 2 * x.numel() * 4 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    for name, dt, n in (("fp64", torch.float64, 8192), ("fp32", torch.float32, 8192),
                        ("bf16", torch.bfloat16, 16384)):
        a = torch.rand(n, n, dtype=torch.float32, device="cuda").to(dt).contiguous()
        b = torch.rand(n, n, dtype=torch.float32, device="cuda").to(dt).contiguous()
        for _ in range(2):
            torch.matmul(a, b)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(3):
            torch.matmul(a, b)
        e1.record()
        torch.cuda.synchronize()
        out[f"{name}_gemm_TFLOPs"] = 2.0 * n ** 3 * 3 / (e0.elapsed_time(e1) * 1e-3) / 1e12
        del a, b
    out["datasheet"] = {"hbm_GBps": 8000.0, "fp64_TFLOPs": FP64_PEAK, "fp32_TFLOPs": FP32_PEAK,
                        "bf16_TFLOPs": BF16_PEAK}
    log("peaks: " + ", ".join(f"{k} {v:.1f}" for k, v in out.items() if not isinstance(v, dict)))
    return out


def qhgk_leg(K, torch, steps, warmup):
    """QHGK conductivity: the 512-atom glass (Eq. qhgk: host FP64
    eigensolver once as set-up, Gamma from the FP32 projection, then the QHGK
    kernels timed; the dense part is 3 (3N)^3 multiply-adds on
    the FP64 matrix cores, of which the tiles on and above the diagonal are
    computed) and the interband term of the perovskite 12^3 mesh
    (Eq. qhgk_crystal) with its RTA conductivity."""
    from synthetic import configs
    out = {}
    c4 = configs.CONFIGS["C4"]
    m4 = configs.model_for(c4)
    cg = K.Crystal.from_model(m4)
    om_h, E_h = K.phonons_gamma(m4.n_basis, m4.mass, m4.fc2)
    om, E = torch.as_tensor(om_h).cuda(), torch.as_tensor(E_h).cuda()
    G = K.linewidths_gamma(cg, om, E, c4.temperature, c4.broadening, K.FP32)
    ws = torch.empty(int(K.lib().kaldo_qhgk_gamma_workspace(cg.handle)), dtype=torch.uint8,
                     device="cuda")
    res = {}

    def step():
        res["k"] = K.qhgk_gamma(cg, m4.frac, om, E, G, c4.temperature, c4.broadening.nu_min_thz,
                                workspace=ws)
    ms, prof = timed(K, torch, step, steps, warmup, "C4 QHGK", plain=True)
    cg.device_status()
    n3 = len(om_h)
    # executed matrix-core work: the tiles on and above the diagonal (the
    # products are symmetric in the mode pair), three components, 2 K FLOP
    # per output element, K = 3N
    nt = (n3 + 63) // 64
    flop = nt * (nt + 1) / 2 * 64 * 64 * 3 * 2.0 * n3
    gemm_ms = prof["qh_gemm"][1] / prof["qh_gemm"][0]
    out["glass"] = dict(modes=n3, ms_per_step=ms, qh_gemm_ms=gemm_ms,
                        kappa_trace_over_3=float(torch.trace(res["k"][0]).item() / 3),
                        roofline=dict(bound="mfma", achieved=flop / (gemm_ms * 1e-3) / 1e12,
                                      peak=FP64_PEAK, unit="TFLOP/s",
                                      frac=flop / (gemm_ms * 1e-3) / 1e12 / FP64_PEAK,
                                      traffic=None, kernel="qh_gemm", flop_per_launch=flop),
                        kernels_ms={k: v[1] / v[0] for k, v in prof.items()})
    cg.close()
    c3 = configs.CONFIGS["C3"]
    m3 = configs.model_for(c3)
    cc = K.Crystal.from_model(m3)
    om3, ev3, ve3 = K.phonons(cc, c3.mesh)
    G3 = K.linewidths(cc, c3.mesh, om3, ev3, ve3, c3.temperature, c3.broadening, K.FP32)
    kr = K.kappa_rta(cc, c3.mesh, om3, ve3, G3, c3.temperature, c3.broadening.nu_min_thz)

    def step3():
        res["ki"] = K.qhgk_crystal(cc, c3.mesh, m3.frac, om3, ev3, G3, c3.temperature,
                                   c3.broadening.nu_min_thz)
    ms3, prof3 = timed(K, torch, step3, steps, warmup, "C3 interband", plain=True)
    cc.device_status()
    out["perovskite_interband"] = dict(
        ms_per_step=ms3, kappa_rta_trace_over_3=float(torch.trace(kr).item() / 3),
        kappa_interband_trace_over_3=float(torch.trace(res["ki"]).item() / 3),
        kernels_ms={k: v[1] / v[0] for k, v in prof3.items()})
    cc.close()
    return out


def isotope_leg(K, torch, cfg, model, c, steps, warmup, gamma_anh=None):
    """Isotope scattering (Eq. isotope) of every mode of the configuration with
    natural compositions: the kernel time, the work it must do (per mode, the
    physical partners inside their cut, counted on the host by interval
    stabbing; per partner 8 (3N_b) + 5 N_b + 10 FLOP: the complex overlaps
    on each atom, their weighted squares and the smearing) against the FP64
    peak, and the conductivity with gamma_iso added to the anharmonic Gamma."""
    from synthetic import configs
    mesh = cfg.mesh
    om, ev, ve = K.phonons(c, mesh)
    g = configs.natural_g(cfg.builder)
    b = cfg.broadening
    ws = torch.empty(K.isotope_workspace(c, mesh), dtype=torch.uint8, device="cuda")
    out = torch.empty(om.shape, dtype=torch.float64, device="cuda")

    def step():
        K.isotope_linewidths(c, mesh, om, ev, ve, g, b, out=out, workspace=ws)
    ms, prof = timed(K, torch, step, steps, warmup, f"{cfg.name} isotope", plain=True)
    c.device_status()
    w = om.cpu().numpy().reshape(-1)
    v = ve.cpu().numpy().reshape(-1, 3)
    phys = w / (2 * np.pi) >= b.nu_min_thz
    if b.adaptive:
        steps2 = np.linalg.inv(np.asarray(model.lattice, float)).T * 2 * np.pi / np.asarray(mesh)[:, None]
        h2 = float(np.sum(steps2 * steps2) / 3.0)
        sig = np.maximum(np.sqrt(np.sum(v * v, axis=1) * h2 / 12.0), 2 * np.pi * b.sigma_floor_thz)
    else:
        sig = np.full(w.shape, 2 * np.pi * b.sigma_thz)
    lo = np.sort((w - 2 * sig)[phys])
    hi = np.sort((w + 2 * sig)[phys])
    wp = w[phys]
    passing = float(np.sum(np.searchsorted(lo, wp, "left") - np.searchsorted(hi, wp, "right")))
    nb = model.n_basis
    flop = passing * (8 * 3 * nb + 5 * nb + 10)
    k_ms = prof["iso_kernel"][1] / prof["iso_kernel"][0]
    res = dict(ms_per_step=ms, iso_kernel_ms=k_ms, g_factor=g, passing_partners=passing,
               roofline=dict(bound="alu", achieved=flop / (k_ms * 1e-3) / 1e12, peak=FP64_PEAK,
                             unit="TFLOP/s", frac=flop / (k_ms * 1e-3) / 1e12 / FP64_PEAK,
                             traffic=None, kernel="iso_kernel", flop_per_launch=flop),
               gamma_iso_max=float(out.max()), kernels_ms={k: v[1] / v[0] for k, v in prof.items()})
    if gamma_anh is not None:
        tot = gamma_anh.clone()
        K.isotope_linewidths(c, mesh, om, ev, ve, g, b, out=tot, accumulate=True, workspace=ws)
        k0 = K.kappa_rta(c, mesh, om, ve, gamma_anh, cfg.temperature, b.nu_min_thz).cpu().numpy()
        k1 = K.kappa_rta(c, mesh, om, ve, tot, cfg.temperature, b.nu_min_thz).cpu().numpy()
        res["kappa_trace_over_3_anharmonic"] = float(np.trace(k0) / 3)
        res["kappa_trace_over_3_with_isotopes"] = float(np.trace(k1) / 3)
    return res


def wedge_leg(K, torch, name, prec, steps, warmup):
    """The irreducible wedge against the full mesh on one configuration (its
    own adaptive smearing): linewidths of the representatives' modes plus the
    star map, against every mode; step times, speedup and the conductivity
    difference (the adaptive widths of degenerate partners follow a gauge
    that is not point-symmetric)."""
    from paper_2602_23728_amd import learned as L
    from synthetic import configs
    cfg = configs.CONFIGS[name]
    model = configs.model_for(cfg)
    c = K.Crystal.from_model(model)
    mesh = cfg.mesh
    nq = int(np.prod(mesh))
    om, ev, ve = K.phonons(c, mesh)
    w = L.Wedge(model.lattice, model.frac, model.mass, mesh)
    ws = torch.empty(max(1, K.linewidths_workspace(c, mesh, prec)), dtype=torch.uint8, device="cuda")
    full = torch.empty(nq, c.nb3, dtype=torch.float64, device="cuda")
    sub = torch.from_numpy(w.rep_modes(c.nb3)).cuda()
    g_ir = torch.zeros(nq, c.nb3, dtype=torch.float64, device="cuda")
    g_w = torch.empty_like(g_ir)

    def s_full():
        K.linewidths(c, mesh, om, ev, ve, cfg.temperature, cfg.broadening, prec, workspace=ws,
                     out=full)

    def s_wedge():
        K.linewidths(c, mesh, om, ev, ve, cfg.temperature, cfg.broadening, prec, subset=sub,
                     workspace=ws, out=g_ir)
        K.star_map(mesh, c.nb3, w.ir_dev, om, g_ir, out=g_w)
    ms_f, _ = timed(K, torch, s_full, steps, warmup, f"{name} full mesh", plain=True)
    ms_w, _ = timed(K, torch, s_wedge, steps, warmup, f"{name} wedge", plain=True)
    kf = K.kappa_rta(c, mesh, om, ve, full, cfg.temperature, cfg.broadening.nu_min_thz).cpu().numpy()
    kw = K.kappa_rta(c, mesh, om, ve, g_w, cfg.temperature, cfg.broadening.nu_min_thz).cpu().numpy()
    c.device_status()
    c.close()
    return dict(irreducible_q=int(w.n_ir), q_points=nq, full_ms=ms_f, wedge_ms=ms_w,
                speedup=ms_f / ms_w, kappa_rel_diff=kappa_rel(kw, kf),
                precision={K.FP64: "fp64", K.FP32: "fp32"}[prec])


def bench_gamma_point(a, cfg, model, K, torch):
    """--config C4 alone: the Gamma-point leg as the JSON line."""
    leg = gamma_point_leg(a, K, torch, cfg, model, a.steps, a.warmup)
    r = leg["bf16x3" if a.precision == "bf16x3" else "fp32"]
    split = a.precision == "bf16x3"
    roof = dict(bound="mfma", achieved=r["gemm_tflops"], peak=r["peak"], unit="TFLOP/s",
                frac=r["gemm_frac"], traffic=None, kernel="gm_gemm",
                work_model="live tiles" + (" (three bf16 products counted)" if split else ""),
                projection_frac=r["projection_frac"])
    print(json.dumps({"metric": METRIC, "value": r["modes_per_s"], "unit": "modes/s",
                      "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
                      "ms_per_step": r["ms_per_step"], "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None,
                      "dtype": "bf16x3" if split else "f32", "data": "synthetic",
                      "config": {"workload": f"{cfg.name}: {cfg.description}",
                                 "modes": leg["modes"], "precision": a.precision},
                      "roofline": roof, "gamma_point": leg}))


def bench_learned(a, cfg, model, c, K, torch):
    """The learned form on a crystal mesh, against the plain FP32 path on every
    mode (the conductivity reference) and on the irreducible wedge."""
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
        state["k"] = kap.clone()

    def ibz():
        om, ev, ve = K.phonons(c, mesh)
        g = L.plain_ibz_linewidths(c, wedge, om, ev, ve, T, b, K.FP32)
        K.kappa_rta(c, mesh, om, ve, g, T, b.nu_min_thz, out=kap)
        state["k"] = kap.clone()

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
        state["k"] = kap.clone()

    ms_full, p_full = timed(K, torch, full, a.steps, a.warmup, "plain-full", plain=True)
    k_full = state["k"].cpu().numpy()
    ms_ibz, p_ibz = timed(K, torch, ibz, a.steps, a.warmup, "plain-wedge", plain=True)
    k_ibz = state["k"].cpu().numpy()
    ms_lrn, p_lrn = timed(K, torch, learned, a.steps, a.warmup, "learned", plain=True)
    k_lrn = state["k"].cpu().numpy()
    res = state["res"]

    def rel(k):
        kbar = np.trace(k_full) / 3
        return float(max(abs(np.trace(k) / 3 - kbar) / kbar, np.max(np.abs(k - k_full)) / kbar))

    n_modes = nq * nb3
    n_rest = len(state["cand"]) - res.n_train - res.n_held
    per = lambda p: {kk: v[1] / a.steps for kk, v in p.items()}  # noqa: E731
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
        "kernels_ms_per_step": {"plain_full": per(p_full), "plain_wedge": per(p_ibz),
                                "learned": per(p_lrn)},
    }))


def kappa_rel(k, ref):
    kbar = np.trace(ref) / 3
    return float(max(abs(np.trace(k) / 3 - kbar) / kbar, np.max(np.abs(k - ref)) / kbar))


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
    if cfg.mesh == (1, 1, 1):
        return bench_gamma_point(a, cfg, model, K, torch)
    c = K.Crystal.from_model(model)
    if a.form == "learned":
        bench_learned(a, cfg, model, c, K, torch)
        c.close()
        return
    if a.form == "qhgk":
        c.close()
        leg = qhgk_leg(K, torch, a.steps, a.warmup)
        g = leg["glass"]
        print(json.dumps({"metric": METRIC, "value": g["modes"] / (g["ms_per_step"] * 1e-3),
                          "unit": "modes/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
                          "ms_per_step": g["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic",
                          "config": {"workload": "C4 glass QHGK and C3 interband term"},
                          "qhgk": leg}))
        return
    if a.form == "isotope":
        leg = isotope_leg(K, torch, cfg, model, c, a.steps, a.warmup)
        n_m = int(np.prod(cfg.mesh)) * c.nb3
        print(json.dumps({"metric": METRIC, "value": n_m / (leg["ms_per_step"] * 1e-3),
                          "unit": "modes/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
                          "ms_per_step": leg["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic",
                          "config": {"workload": f"{cfg.name} isotope scattering"},
                          "isotope": leg}))
        c.close()
        return
    if a.form == "tsweep":
        step, bufs = crystal_step(K, torch, c, cfg, K.FP64)
        step()
        torch.cuda.synchronize()
        leg = tsweep_leg(K, torch, cfg, model, c, a.steps, a.warmup, direct_gamma=bufs["gam"])
        print(json.dumps({"metric": METRIC,
                          "value": leg["modes_temperatures_per_s"], "unit": "mode-temperatures/s",
                          "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
                          "ms_per_step": leg["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic",
                          "config": {"workload": f"{cfg.name} temperature sweep from the cache"},
                          "tsweep": leg}))
        c.close()
        return
    if a.form == "bte":
        c.close()
        leg = bte_leg(K, torch, a.steps, a.warmup)
        print(json.dumps({"metric": METRIC, "value": leg["modes"] / (leg["ms_per_step"] * 1e-3),
                          "unit": "modes/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
                          "ms_per_step": leg["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic",
                          "config": {"workload": "C2 full BTE: scattering matrix and inverse"},
                          "bte_c2": leg}))
        return
    mesh = cfg.mesh
    nq = int(np.prod(mesh))
    nb3 = c.nb3
    n_modes = nq * nb3

    step, bufs = crystal_step(K, torch, c, cfg, prec)
    ms_per_step, prof = timed(K, torch, step, a.steps, a.warmup, f"{cfg.name} {a.precision}")
    c.device_status()  # raises if a kernel found invalid inputs
    kappa = bufs["kap"].cpu().numpy()
    dom, (launches, total) = max(prof.items(), key=lambda kv: kv[1][1])
    avg_ms = total / launches

    extras = {}
    if not a.no_extras:
        if prec != K.FP32:
            step32, b32 = crystal_step(K, torch, c, cfg, K.FP32)
            ms32, prof32 = timed(K, torch, step32, a.steps, a.warmup, f"{cfg.name} fp32", plain=True)
            k32 = b32["kap"].cpu().numpy()
            extras["fp32"] = dict(ms_per_step=ms32, modes_per_s=n_modes / (ms32 * 1e-3),
                                  speedup_vs_headline=ms_per_step / ms32,
                                  kappa_rel_diff_vs_headline=kappa_rel(k32, kappa),
                                  kernels_ms={k: v[1] / v[0] for k, v in prof32.items()})
            del b32
        # split precision against plain FP32 on the perovskite 12^3 mesh
        c3 = configs.CONFIGS["C3"]
        m3 = configs.model_for(c3)
        cc3 = K.Crystal.from_model(m3)
        n3 = int(np.prod(c3.mesh)) * cc3.nb3
        leg = {}
        ks = {}
        for name, p in (("fp32", K.FP32), ("bf16x3", K.BF16X3)):
            s3, b3 = crystal_step(K, torch, cc3, c3, p)
            ms3, pr3 = timed(K, torch, s3, max(3, a.steps // 4), 2, f"C3 {name}", plain=True)
            ks[name] = b3["kap"].cpu().numpy()
            leg[name] = dict(ms_per_step=ms3, modes_per_s=n3 / (ms3 * 1e-3),
                             kernels_ms={k: v[1] / v[0] for k, v in pr3.items()})
            del b3
        cc3.device_status()
        leg["split_speedup"] = leg["fp32"]["ms_per_step"] / leg["bf16x3"]["ms_per_step"]
        leg["kappa_rel_diff_split_vs_fp32"] = kappa_rel(ks["bf16x3"], ks["fp32"])
        cc3.close()
        extras["c3_split"] = leg
        c4 = configs.CONFIGS["C4"]
        extras["c4"] = gamma_point_leg(a, K, torch, c4, configs.model_for(c4),
                                       max(3, a.steps // 4), 2)
        extras["bte_c2"] = bte_leg(K, torch, 3, 1)
        extras["qhgk"] = qhgk_leg(K, torch, max(3, a.steps // 4), 1)
        extras["peaks"] = peaks_leg(torch)
        extras["isotope"] = isotope_leg(K, torch, cfg, model, c, max(3, a.steps // 4), 1,
                                        gamma_anh=bufs["gam"])
        extras["wedge"] = {"C2": wedge_leg(K, torch, "C2", K.FP64, max(3, a.steps // 4), 1),
                           "C3": wedge_leg(K, torch, "C3", K.FP32, max(3, a.steps // 4), 1)}
        if prec == K.FP64:
            leg = tsweep_leg(K, torch, cfg, model, c, max(3, a.steps // 4), 1,
                             direct_gamma=bufs["gam"])
            # per temperature, against the direct path's projection kernel
            leg["speedup_per_temperature_vs_direct"] = avg_ms / leg["ms_per_temperature"]
            extras["tsweep"] = leg

    base, stats, om_o = (None, {}, None)
    if not a.no_cpu_baseline:
        base, stats, om_o = cpu_baseline(cfg, model, a.cpu_seconds)
        log(f"cpu baseline {base['value']:.1f} modes/s ({base['sample']})")
    roof = None
    if dom in ("lw_crystal", "lw_fused") and stats:
        w = pruned_work(model, nq, stats, om_o, cfg.broadening.nu_min_thz)
        fp64 = prec == K.FP64
        peak = FP64_PEAK if fp64 else FP32_PEAK
        achieved = w["total_flop"] / (avg_ms * 1e-3) / 1e12
        # With Phi3 symmetric in its last two slots the fused kernel visits each
        # mirrored partner pair (q1, q2) once: on average (N_q + 1) / 2 partner
        # points per q, about half of the ordered-pair work counted above.
        f_exec = (nq + 1) / (2.0 * nq) if (dom == "lw_fused" and fc3_mirror_symmetric(model)) else 1.0
        roof = dict(bound="alu", achieved=achieved, peak=peak, unit="TFLOP/s",
                    frac=achieved / peak, traffic=measured_traffic(dom, cfg.name, a.precision),
                    kernel=dom, kernel_ms=avg_ms,
                    work_model="pruned, ordered partner pairs, physical modes "
                               "(8 N_q (f_blk n_p + f_pass nb3^4) FLOP each)",
                    flop_per_mode=w["flop_per_mode"], physical_modes=w["physical_modes"],
                    f_blk=w["f_blk"], f_pass=w["f_pass"], executed_fraction=f_exec,
                    executed_tflops=achieved * f_exec, executed_frac=achieved * f_exec / peak,
                    dense_equiv_tflops=w["dense_flop_per_mode"] * w["physical_modes"]
                    / (avg_ms * 1e-3) / 1e12)
    if dom.startswith("lw_mfma"):
        # Dense MFMA kernel: per (q, swept partner q1, live branch s) two complex
        # 16x16x16 products (T = B_s eta2, V = eta1^T T), each two real 16x16x32
        # products, i.e. 65,536 FLOP; the BF16x3 form issues three BF16 products
        # per real product.  Partners: (N_q + 1) / 2 per q on average when the
        # mirrored pair is visited once, else N_q.
        om_h = bufs["om"].cpu().numpy()
        n_live = int(np.sum(om_h / (2 * np.pi) >= cfg.broadening.nu_min_thz))
        partners = (nq + 1) / 2.0 if fc3_mirror_symmetric(model) else float(nq)
        split = prec == K.BF16X3
        flop = n_live * partners * 65536.0 * (3 if split else 1)
        achieved = flop / (avg_ms * 1e-3) / 1e12
        peak = BF16_PEAK if split else FP32_PEAK
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
    out.update(extras)
    c.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
