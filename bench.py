#!/usr/bin/env python3
"""Benchmark of the LOBPCG-F hot path on one MI355X.

Workload (the headline): the heavy-dimer system (cubic 20 bohr cell, Gamma
point, Ecut 30 Ha, 62 669 planewaves x 4 components, 96^3 FFT grid,
c = 137.036, 40 bands, Gaussian local potentials of depth -80 Ha / width
0.4 bohr, l = 0..2 spin-orbit projectors with two radial functions), seeded
synthetic inputs, seeds 0, 1 and 2 (median reported).

A step is one LOBPCG-F iteration of Algorithm 1 on the 40-band block in FP64:
the filter (two H applications), H Y, the Gram products of [X, Y, P], the FP64
Rayleigh-Ritz, the block updates and the residual norms.  W warm-up iterations
and then exactly K timed iterations run inside one solve whose tolerance is
set below reach, so every column stays active and every step does the full
work; each iteration ends with a stream synchronisation and its wall time is
recorded by the library.  The JSON line also reports H.X throughput, the mixed
FP32 iteration rate, time to a 1e-8 Ha solution in FP64 and in mixed precision
with per-band errors against the oracle's golden values, the tiny dimer
(iterations/s and time to solution), the 64-system uneven batch, the 16
k-points of the layered crystal solved to 1e-8 Ha, the roofline of the
dominant kernel, and the FP64 CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 (vector = matrix)
FP32_PEAK_TFLOPS = 157.3        # FP32 matrix (dense)
BF16_PEAK_TFLOPS = 2500.0       # BF16 matrix (dense)


def ip_pairs(nz, tile=64):
    """(i, j) output pairs of the Hermitian Gram kernel: the 64 x 64 tiles on and
    above the diagonal of an nz x nz product, clipped at nz."""
    t = (nz + tile - 1) // tile
    size = [min(tile, nz - a * tile) for a in range(t)]
    return sum(size[a] * size[b] for a in range(t) for b in range(a, t))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic(kernel, s, N, ncol, nrows, nb):
    """Algorithmic HBM bytes and flops of one launch of `kernel` on nb bands.

    Bytes -- k_plane: each (band-component, z plane) reads and writes its ncol
    pruned column values once, and the local potential is read once per
    launch; k_zfft_inv / k_zfft_fwd: the sphere block (read, or read + write for
    the accumulate) plus the pruned column block.
    Flops -- the nominal 5 n log2 n of a length-n complex FFT per line: k_plane
    transforms nrows lines along a2 and n2 lines along a1, each inverse and
    forward, plus 2 flops per point for the real potential; the z transforms
    one line of n3 per column.  Returns (bytes, flops) or (None, None)."""
    n1, n2, n3 = s.grid
    cs = 16 if kernel.endswith(".f64") else 8
    rs = cs // 2
    ncols = 4 * nb
    f1, f2, f3 = (5 * m * math.log2(m) for m in (n1, n2, n3))
    if kernel.startswith("k_plane"):
        by = ncols * n3 * 2 * ncol * cs + n1 * n2 * n3 * rs
        fl = ncols * n3 * (2 * nrows * f2 + 2 * n2 * f1 + 2 * n1 * n2)
        return by, fl
    if kernel.startswith("k_zfft_inv"):
        return ncols * (N + n3 * ncol) * cs, ncols * ncol * f3
    if kernel.startswith("k_zfft_fwd"):
        return ncols * (2 * N + n3 * ncol) * cs, ncols * ncol * f3
    return None, None


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy), or None when there is
    no summary for it or its sources changed since the counters were taken."""
    import hashlib
    name = kernel.replace(".", "_")
    path = os.path.join(ROOT, "profiles", f"{name}_heavy_dimer_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    h = hashlib.sha256()
    for f in d["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != d["sources_sha256"]:
        return None
    return d["traffic_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-solution runs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-solve runs")
    ap.add_argument("--only-scf", action="store_true",
                    help="profiling aid: only the heavy-dimer SCF loops (DKS and KSSO)")
    ap.add_argument("--only-layered", action="store_true",
                    help="profiling aid: only the layered crystal's batched solves and its "
                         "all-active k-point iteration")
    ap.add_argument("--only-apply", action="store_true",
                    help="profiling aid: only K FP64 H.X applications of the 40-band block, then "
                         "one device copy of 1 GiB (the calibration kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(every system is solved on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    K, W = args.steps, args.warmup

    # sixteen hardware queues (HIP's default is four): the batched solves run
    # two lanes per queue; must be set before the HIP runtime starts
    os.environ["GPU_MAX_HW_QUEUES"] = "16"
    import numpy as np
    import torch

    import paper_1211_1446_amd as dk
    import sysgen

    dev = torch.device("cuda:0")
    t0 = time.time()
    s = sysgen.heavy_dimer(0)
    b = dk.init_basis([s])
    N, grid, mil = dk.basis_info(b, 0)
    n = s.n_bands
    log(f"[bench] heavy dimer: N={N} grid={grid} n={n} setup {time.time() - t0:.1f}s")
    ncol = len({(int(a), int(c)) for a, c in mil[:, :2]})
    nrows = len({int(a) for a in mil[:, 0]})

    phi = sysgen.start_block(mil, s.lattice, s.kpts[0], n, 0)
    X0 = np.zeros((n, 4, N), dtype=np.complex128)
    X0[:, :2] = phi
    X0d = torch.from_numpy(X0).to(dev)
    stream = torch.cuda.current_stream()

    def golden_of(name):
        path = os.path.join(ROOT, "tests", "golden", name)
        return json.load(open(path)) if os.path.exists(path) else None

    # ---- the layered crystal: the 16 k-points of 120 bands (N ~ 17.0k each,
    # 48 x 48 x 320 grid) solved to 1e-8 Ha in one batched call, FP64 and
    # mixed; per-band errors of k-point 0 and its partner -k (k-point 15)
    # against the oracle's golden; the all-active FP64 iteration on one k-point
    def run_layered():
        sL = sysgen.layered_crystal(0)
        bL = dk.init_basis([sL])
        nkL = sL.kpts.shape[0]
        gL = golden_of("layered_crystal_seed0_k0.json")
        nwL = sL.n_bands
        # 40 buffer columns (n_Z = 480): 598 k-point iterations instead of 2 403 with 8, and
        # the shortest time to solution of 8, 16, 24 and 40 (each k-point's Rayleigh-Ritz
        # grows with n_Z, but the 16 run concurrently)
        bufL = 40
        nL = nwL + bufL
        XsL, npwL = [], []
        for i in range(nkL):
            NL, _, milL = dk.basis_info(bL, i)
            X0L = np.zeros((nL, 4, NL), dtype=np.complex128)
            X0L[:, :2] = sysgen.start_block(milL, sL.lattice, sL.kpts[i], nL, i)
            XsL.append(torch.from_numpy(X0L).to(dev))
            npwL.append(NL)
        layered = {"kpoints": nkL, "npw_per_k": npwL, "bands": nwL, "buffer_columns": bufL,
                   "grid": list(sL.grid)}
        for tag, mode in (("fp64", dk.MODE_FP64), ("mixed_fp32", dk.MODE_MIXED_FP32)):
            o = dk.default_opts(mode=mode, tol=1e-8, n_iter=400, kinetic_balance=1, n_buffer=bufL)
            Xw = [x.clone() for x in XsL]
            torch.cuda.synchronize()
            t = time.perf_counter()
            lams, _, infos, _ = dk.lobpcgf_solve_batch(bL, list(range(nkL)), [nL] * nkL, Xw, o)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            its = sum(i_["iterations"] for i_ in infos)
            rec = {"seconds": dt, "converged": sum(int(i_["converged"]) for i_ in infos),
                   "kpoint_iterations": its, "kpoint_iterations_per_s": its / dt,
                   "worst_resnorm": max(i_["max_resnorm"] for i_ in infos),
                   "iterations_per_k": [i_["iterations"] for i_ in infos]}
            if gL:
                ref = np.array(gL["eigenvalues"])   # the lowest len(ref) of the 120
                for kk in (0, nkL - 1):
                    err = np.abs(np.asarray(lams[kk][:len(ref)]) - ref)
                    rec[f"k{kk}_max_abs_err_vs_oracle_Ha"] = float(err.max())
                    rec[f"k{kk}_per_band_err_Ha"] = [float(x) for x in err]
            layered[f"{tag}_to_1e-8"] = rec
            log(f"[bench] layered crystal {tag}: 16 k to 1e-8 in {dt:.2f}s "
                f"({rec['converged']}/16 converged, {its} k-point iterations)")
        layered["mixed_fp32_speedup_vs_fp64"] = (layered["fp64_to_1e-8"]["seconds"] /
                                                 layered["mixed_fp32_to_1e-8"]["seconds"])
        it64 = np.zeros(16)
        o64 = dk.default_opts(tol=1e-300, n_iter=4, kinetic_balance=1)
        dk.lobpcgf_solve(bL, 0, nwL, XsL[0][:nwL].clone(), o64, iter_ms=it64)
        layered["fp64_kpoint_iteration_ms_120_bands"] = float(np.mean(it64[1:4]))
        bL.close()
        return layered

    # ---- the SCF loop around the eigensolver (Sec. 4; Table 6 reports the wall
    # time per SCF step): 24 electrons in the 40 lowest bands (+ 8 buffer
    # columns) at 5000 K, 5 eigensolver iterations per step, Anderson + Kerker
    # mixing, to ||dV|| / ||V|| < 1e-8 with every wanted residual below 1e-8;
    # DKS (LOBPCG-F) and KSSO (standard LOBPCG)
    def run_scf():
        v_ext = dk.get_local_potential(b, 0).clone()
        nscf = n + 8
        phis = sysgen.start_block(mil, s.lattice, s.kpts[0], nscf, 0)
        X4s = np.zeros((nscf, 4, N), dtype=np.complex128)
        X4s[:, :2] = phis
        scf_rec = {"workload": "heavy dimer, 24 electrons in the 40 lowest bands + 8 buffer at "
                               "5000 K, 5 eigensolver iterations (Teter-preconditioned) per SCF "
                               "step, Anderson + Kerker, tol 1e-8", "models": {}}
        for tag, model, start in (("dks", dk.MODEL_DKS, X4s), ("ksso", dk.MODEL_KSSO, phis)):
            dk.set_local_potential(b, 0, v_ext)
            Xs = torch.from_numpy(np.ascontiguousarray(start)).to(dev)
            eo = dk.default_opts(model=model, kinetic_balance=1 if model == dk.MODEL_DKS else 0,
                                 use_filter=1 if model == dk.MODEL_DKS else 0, tol=1e-8, n_buffer=8,
                                 n_iter=400)
            so = dk.scf_default_opts(n_electrons=24.0, tol=1e-8, max_scf=120, eig_iters=5)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, occ_, info_, rc_ = dk.scf(b, 0, nscf, Xs, so, eo)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t
            scf_rec["models"][tag] = {
                "seconds": sec, "steps": info_["iterations"],
                "step_ms": 1000.0 * sec / max(info_["iterations"], 1),
                "ms_per_eig_iteration": 1000.0 * sec / max(info_["eig_iterations"], 1),
                "eig_iterations": info_["eig_iterations"], "converged": info_["converged"],
                "status": rc_, "residual": info_["residual"], "free_energy_Ha": info_["free_energy"],
                "fermi_Ha": info_["fermi"], "max_bxc_Ha": info_["max_bxc"]}
            log(f"[bench] SCF {tag}: {info_['iterations']} steps in {sec:.3f}s "
                f"({1000.0 * sec / max(info_['iterations'], 1):.2f} ms/step), converged {info_['converged']}, "
                f"residual {info_['residual']:.1e}")
        m_ = scf_rec["models"]
        scf_rec["dks_over_ksso_step_cost"] = m_["dks"]["step_ms"] / m_["ksso"]["step_ms"]
        dk.set_local_potential(b, 0, v_ext)
        return scf_rec

    if args.only_scf:
        run_scf()
        b.close()
        return

    if args.only_layered:
        run_layered()
        b.close()
        return

    if args.only_apply:
        Xd = X0d
        HXd = torch.empty_like(Xd)
        for _ in range(W + K):
            dk.apply_H(b, 0, Xd, HXd)
        big = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        big.fill_(1.0)
        dst = torch.empty_like(big)
        torch.cuda.synchronize()
        dst.copy_(big)
        torch.cuda.synchronize()
        log(f"[bench] only-apply: {W + K} FP64 applies of {n} bands, 1 GiB copy")
        b.close()
        return

    # ---- H.X throughput, FP64 and FP32 (whole 40-band block per call)
    hx = {}
    for tag, ctype in (("fp64", torch.complex128), ("fp32", torch.complex64)):
        Xd = X0d.to(ctype)
        HXd = torch.empty_like(Xd)
        for _ in range(W):
            dk.apply_H(b, 0, Xd, HXd)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(K):
            dk.apply_H(b, 0, Xd, HXd)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        hx[tag] = {"ms_per_apply": ms, "spinor_bands_per_s": n / (ms * 1e-3)}
        log(f"[bench] apply_H {tag}: {ms:.3f} ms / {n} bands")

    # ---- per-kernel live timing of the FP64 apply (events on the launch stream)
    Xd = X0d
    HXd = torch.empty_like(Xd)
    dk.profile_enable(True)
    for _ in range(K):
        dk.apply_H(b, 0, Xd, HXd)
    kstats = dk.profile_report()
    dk.profile_enable(False)
    kernels = {k: {"count": v["count"], "avg_ms": v["total_ms"] / v["count"]} for k, v in kstats.items()}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["count"])
    by, fl = algorithmic(dom, s, N, ncol, nrows, n)
    roof = None
    if by is not None:
        # the binding roofline is the one whose ideal time is longer: HBM bytes at
        # 8 TB/s or FP64 vector flops at 78.6 TFLOP/s (FFT arithmetic, no MFMA)
        t = kernels[dom]["avg_ms"] * 1e-3
        gbs, tfs = by / t / 1e9, fl / t / 1e12
        alu = fl / (FP64_PEAK_TFLOPS * 1e12) > by / (HBM_PEAK_GBS * 1e9)
        roof = {"kernel": dom, "bound": "alu" if alu else "hbm",
                "achieved": tfs if alu else gbs,
                "peak": FP64_PEAK_TFLOPS if alu else HBM_PEAK_GBS,
                "unit": "TFLOP/s" if alu else "GB/s",
                "frac": tfs / FP64_PEAK_TFLOPS if alu else gbs / HBM_PEAK_GBS,
                "traffic": measured_traffic(dom),
                "algorithmic_bytes_per_launch": by, "algorithmic_flops_per_launch": fl,
                "hbm_GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                "fp64_TFLOPs": tfs, "fp64_frac": tfs / FP64_PEAK_TFLOPS,
                "avg_launch_ms": kernels[dom]["avg_ms"]}
    log(f"[bench] kernels: " + ", ".join(f"{k} {v['avg_ms']:.3f}ms" for k, v in kernels.items()))

    # ---- LOBPCG-F iterations (FP64), all columns active
    def iterations(mode, nit):
        Xd = X0d.clone()
        it_ms = np.zeros(nit + (nit if mode else 0) + 4)
        if mode == dk.MODE_FP64:
            o = dk.default_opts(tol=1e-300, n_iter=nit, kinetic_balance=1)
        else:
            o = dk.default_opts(mode=mode, tol=1e-300, n_iter=0, mixed_iter=nit,
                                mixed_tol=-1.0, kinetic_balance=1)
        lam, res, info, rc = dk.lobpcgf_solve(b, 0, n, Xd, o, iter_ms=it_ms)
        return it_ms, info

    # ---- matrix-core kernels of one full iteration (n_Z = 3n, every column active):
    # per-launch times from two profiled runs (2 and 8 iterations) differenced, so
    # that only full-size launches remain; algorithmic flops 8 per complex MAC
    # (the FP32 Gram's three-product form does 6 real flops per MAC of useful work)
    def profiled(mode, nit):
        dk.profile_enable(True)
        iterations(mode, nit)
        rep_ = dk.profile_report()
        dk.profile_enable(False)
        return rep_
    K4 = 4 * N
    nz = 3 * n
    nproj = sum(g.n_rad * (2 * g.l + 1) for g in s.proj)   # scalar projectors (B has nproj rows)
    mk = {}
    for mode, sfx, peak in ((dk.MODE_FP64, "f64", FP64_PEAK_TFLOPS),
                            (dk.MODE_MIXED_FP32, "f32", FP32_PEAK_TFLOPS),
                            (dk.MODE_MIXED_BF16GRAM, "bf16", BF16_PEAK_TFLOPS)):
        a, c = profiled(mode, 2), profiled(mode, 8)
        # the Gram pair S = Z^H Z, A = Z^H H Z: one fused launch (BF16-split), or
        # S and A as launches of their own (the unbatched solver forms S before
        # H Y): its flops are per iteration and shared among the launches seen
        per_it = {
            f"k_gemm_ip.gram.{sfx}": (None, 8.0 * 2 * ip_pairs(nz) * K4),
            # X and H X (m = n_Z rows), P and H P (2n rows): one paired launch each
            f"k_gemm_up.{sfx}": (2, 8.0 * K4 * n * (2 * nz + 2 * (2 * n)) / 2),
            f"k_gemm_ip.{sfx}": (3, 8.0 * nproj * 4 * n * N),
        }
        for kname, spec in per_it.items():
            if spec is None or kname not in c or kname not in a:
                continue
            launches, flops = spec
            cnt = c[kname]["count"] - a[kname]["count"]
            tot = c[kname]["total_ms"] - a[kname]["total_ms"]
            if cnt <= 0 or tot <= 0:
                continue
            ms = tot / cnt
            if launches is None:
                flops = flops / (cnt / 6.0)
            tf = flops / (ms * 1e-3) / 1e12
            kp = peak if sfx != "bf16" or "gram" in kname else FP32_PEAK_TFLOPS
            mk[kname] = {"avg_ms": ms, "launches_per_iteration": cnt / 6.0,
                         "algorithmic_gflop_per_launch": flops / 1e9, "tflops": tf,
                         "peak_tflops": kp, "frac": tf / kp}
            if ".gram." in kname:
                # the same launch counted on the unique entries of the Hermitian
                # products (j >= i) instead of the computed upper tiles
                uf = tf * (nz * (nz + 1) / 2) / ip_pairs(nz)
                mk[kname]["unique_entry_tflops"] = uf
                mk[kname]["unique_entry_frac"] = uf / kp
    log("[bench] matrix kernels: " + ", ".join(f"{k} {v['tflops']:.1f} TF/s ({100 * v['frac']:.0f} %)"
                                              for k, v in mk.items()))

    it_ms, info64 = iterations(dk.MODE_FP64, W + K)
    per_seed_ms = {0: float(np.mean(it_ms[W:W + K]))}
    log(f"[bench] FP64 LOBPCG-F iteration, seed 0: {per_seed_ms[0]:.3f} ms")
    it32, info32 = iterations(dk.MODE_MIXED_FP32, W + K)
    step32_ms = float(np.mean(it32[W:W + K]))
    log(f"[bench] FP32 LOBPCG-F iteration: {step32_ms:.3f} ms")

    def solve_record(bs, nb, X0_, mode, ref=None, n_buffer=0, method=None):
        Xd_ = X0_.clone()
        o = dk.default_opts(mode=mode, tol=1e-8, n_iter=400, kinetic_balance=1, n_buffer=n_buffer,
                            method=dk.METHOD_LOBPCG if method is None else method)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lam, res, info, rc = dk.lobpcgf_solve(bs, 0, nb, Xd_, o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        rec = {"seconds": dt, "iterations": info["iterations"],
               "iters_reduced": info["iters_reduced"], "status": rc,
               "max_resnorm": info["max_resnorm"], "h_band_applies": info["h_applies"]}
        if ref is not None:
            nw = nb - n_buffer
            err = np.abs(np.asarray(lam[:nw]) - np.asarray(ref[:nw]))
            rec["max_abs_err_vs_oracle_Ha"] = float(err.max())
            rec["per_band_err_Ha"] = [float(x) for x in err]
        return rec

    MODES = (("fp64", dk.MODE_FP64), ("mixed_fp32", dk.MODE_MIXED_FP32),
             ("mixed_bf16gram", dk.MODE_MIXED_BF16GRAM))

    # ---- time to a 1e-8 Ha solution, FP64 vs mixed (FP32 bulk + FP64 polish), seed 0
    tts = {"seeds": {}}
    gh = golden_of("heavy_dimer_seed0.json")
    if not args.no_solve:
        tts["seeds"]["0"] = {}
        for tag, mode in MODES:
            rec = solve_record(b, n, X0d, mode, gh["eigenvalues"] if gh else None)
            tts["seeds"]["0"][tag] = rec
            log(f"[bench] seed 0 solve {tag}: {rec['seconds']:.3f}s, {rec['iterations']} it, "
                f"max|r| {rec['max_resnorm']:.2e}")
        # the filter inside a block Davidson solver (FP64, space of 4n vectors)
        rec = solve_record(b, n, X0d, dk.MODE_FP64, gh["eigenvalues"] if gh else None,
                           method=dk.METHOD_DAVIDSON)
        tts["seeds"]["0"]["davidson_fp64"] = rec
        log(f"[bench] seed 0 solve davidson_fp64: {rec['seconds']:.3f}s, {rec['iterations']} it, "
            f"max|r| {rec['max_resnorm']:.2e}")

    # ---- the paper's comparison module (Table 1): the two-component KSSO
    # operator |k+G|^2/2 + V_loc + V_2 on the same system, standard LOBPCG (one
    # H apply per iteration, no filter), 40 bands; the DKS / KSSO cost ratio
    # (the paper reports x~4 per SCF step: twice the components, three applies)
    ksso = None
    if not args.no_solve:
        Xk = torch.from_numpy(np.ascontiguousarray(phi)).to(dev)     # (n, 2, N)
        itk = np.zeros(W + K + 4)
        dk.lobpcgf_solve(b, 0, n, Xk.clone(), dk.default_opts(model=dk.MODEL_KSSO, tol=1e-300,
                                                                n_iter=W + K), iter_ms=itk)
        ksso_ms = float(np.mean(itk[W:W + K]))
        Xk2 = Xk.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        lamk, _, infok, rck = dk.lobpcgf_solve(b, 0, n, Xk2, dk.default_opts(model=dk.MODEL_KSSO,
                                                                               n_iter=400))
        torch.cuda.synchronize()
        ksso_tts = time.perf_counter() - t
        ksso = {"workload": "heavy dimer, two-component KSSO, standard LOBPCG, 40 bands",
                "iteration_ms": ksso_ms, "iterations_per_s": 1000.0 / ksso_ms,
                "time_to_solution_1e-8_s": ksso_tts, "iterations": infok["iterations"],
                "status": rck,
                "dks_over_ksso_iteration_cost": per_seed_ms[0] / ksso_ms,
                "dks_over_ksso_time_to_solution": (tts["seeds"]["0"]["fp64"]["seconds"] / ksso_tts
                                                   if tts["seeds"] else None)}
        log(f"[bench] KSSO LOBPCG iteration {ksso_ms:.3f} ms, to 1e-8 {ksso_tts:.3f}s "
            f"({infok['iterations']} it); DKS/KSSO per iteration {ksso['dks_over_ksso_iteration_cost']:.2f}")

    scf_rec = run_scf() if not args.no_solve else None
    b.close()

    # ---- seeds 1 and 2 of the same workload: the timed iterations (the
    # headline is the median over seeds 0, 1, 2) and the time to solution
    for seed in (1, 2):
        s_ = sysgen.heavy_dimer(seed)
        b_ = dk.init_basis([s_])
        N_, _, mil_ = dk.basis_info(b_, 0)
        X_ = np.zeros((n, 4, N_), dtype=np.complex128)
        X_[:, :2] = sysgen.start_block(mil_, s_.lattice, s_.kpts[0], n, seed)
        Xs_ = torch.from_numpy(X_).to(dev)
        it_ = np.zeros(W + K + 4)
        dk.lobpcgf_solve(b_, 0, n, Xs_.clone(),
                         dk.default_opts(tol=1e-300, n_iter=W + K, kinetic_balance=1), iter_ms=it_)
        per_seed_ms[seed] = float(np.mean(it_[W:W + K]))
        log(f"[bench] FP64 LOBPCG-F iteration, seed {seed}: {per_seed_ms[seed]:.3f} ms")
        if not args.no_solve:
            tts["seeds"][str(seed)] = {}
            for tag, mode in MODES:
                rec = solve_record(b_, n, Xs_, mode)
                tts["seeds"][str(seed)][tag] = rec
                log(f"[bench] seed {seed} solve {tag}: {rec['seconds']:.3f}s, "
                    f"{rec['iterations']} it, max|r| {rec['max_resnorm']:.2e}")
        b_.close()
    step_ms = float(np.median(list(per_seed_ms.values())))
    if not args.no_solve:
        for tag, _ in MODES:
            tts[f"{tag}_median_s"] = float(np.median([tts["seeds"][k][tag]["seconds"]
                                                      for k in tts["seeds"]]))
        tts["mixed_fp32_speedup_vs_fp64"] = tts["fp64_median_s"] / tts["mixed_fp32_median_s"]

    # ---- the tiny dimer (cubic 10 bohr, Ecut 5 Ha, 24^3, N = 515, 8 bands):
    # all-active FP64 iterations and the time to 1e-8 Ha against the dense oracle
    tiny = None
    if not args.no_solve:
        gt = golden_of("tiny_dimer_seeds.json")
        tiny = {"workload": "tiny_dimer: cubic 10 bohr, Gamma, Ecut 5 Ha, 24^3, 8 bands",
                "seeds": {}}
        for seed in (0, 1, 2):
            st_ = sysgen.tiny_dimer(seed)
            bt = dk.init_basis([st_])
            Nt, _, milt = dk.basis_info(bt, 0)
            Xt = np.zeros((8, 4, Nt), dtype=np.complex128)
            Xt[:, :2] = sysgen.start_block(milt, st_.lattice, st_.kpts[0], 8, seed)
            Xtd = torch.from_numpy(Xt).to(dev)
            itt = np.zeros(W + K + 4)
            dk.lobpcgf_solve(bt, 0, 8, Xtd.clone(),
                             dk.default_opts(tol=1e-300, n_iter=W + K, kinetic_balance=1),
                             iter_ms=itt)
            ref = gt["seeds"][str(seed)]["eigenvalues"] if gt else None
            rec = {"fp64_iteration_ms": float(np.mean(itt[W:W + K]))}
            for tag, mode in MODES[:2]:
                rec[tag] = solve_record(bt, 8, Xtd, mode, ref)
            tiny["seeds"][str(seed)] = rec
            bt.close()
        ms_t = float(np.median([v["fp64_iteration_ms"] for v in tiny["seeds"].values()]))
        tiny["fp64_iterations_per_s_median"] = 1000.0 / ms_t
        tiny["fp64_time_to_solution_median_s"] = float(np.median(
            [v["fp64"]["seconds"] for v in tiny["seeds"].values()]))
        errs = [v[t].get("max_abs_err_vs_oracle_Ha", float("nan"))
                for v in tiny["seeds"].values() for t in ("fp64", "mixed_fp32")]
        tiny["max_abs_err_vs_oracle_Ha"] = float(np.max(errs))
        log(f"[bench] tiny dimer: {tiny['fp64_iterations_per_s_median']:.0f} it/s, "
            f"max error {tiny['max_abs_err_vs_oracle_Ha']:.1e} Ha")

    # ---- batched solves: the 64 uneven independent systems, in one
    # dks_lobpcgf_solve_batch call versus one solve after another
    batch = None
    if not args.no_solve and not args.no_batch:
        systems = sysgen.uneven_batch(seed=0, count=64)
        bb = dk.init_basis(systems)
        # wanted bands per system from the generator, plus kBuf buffer columns
        # (n_buffer: iterated, not required to converge; one value for the whole
        # batch call), the usual LOBPCG practice for spectra whose wanted count
        # falls inside a close group
        # per item about two thirds of the wanted count as buffer columns (at
        # least 8, even): the generator's cubic cells have near-degenerate
        # shells of up to ~2n/3 states at the wanted count (system 27: 18
        # states within 1.6e-3 Ha around its 24th), and a block that ends inside
        # one converges at ~0.99 per iteration
        wanted = [s_.n_bands for s_ in systems]
        bufs = [max(8, ((2 * w_) // 3 + 1) // 2 * 2) for w_ in wanted]
        ns = [w_ + b_ for w_, b_ in zip(wanted, bufs)]
        sizes = [dk.basis_info(bb, i, miller=False)[0] for i in range(len(systems))]
        gd = golden_of("uneven_batch_seed0_dense.json")
        dense = {int(k): np.array(v["eigenvalues"]) for k, v in gd["systems"].items()} if gd else {}

        def blocks():
            Xs = []
            for i, (s_, n_) in enumerate(zip(systems, ns)):
                _, _, mil_ = dk.basis_info(bb, i)
                X0_ = np.zeros((n_, 4, sizes[i]), dtype=np.complex128)
                X0_[:, :2] = sysgen.start_block(mil_, s_.lattice, s_.kpts[0], n_, 100 + i)
                Xs.append(torch.from_numpy(X0_).to(dev))
            return Xs
        batch = {"systems": len(systems), "npw": sizes, "bands": wanted, "buffer_columns": bufs,
                 "systems_with_dense_golden": sorted(dense),
                 "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"])}
        # launch shapes of every system picked by the library's autotuner
        t = time.perf_counter()
        dk.autotune(bb, list(range(len(systems))), ns)
        torch.cuda.synchronize()
        batch["autotune_s"] = time.perf_counter() - t
        batch["tuning"] = [dk.get_tuning(bb, i) for i in range(len(systems))]
        runs = (("fp64", dk.MODE_FP64, 0), ("mixed_fp32", dk.MODE_MIXED_FP32, 0),
                ("fp64_graph", dk.MODE_FP64, 1), ("mixed_fp32_graph", dk.MODE_MIXED_FP32, 1))
        for tag, mode, graph in runs:
            o = dk.default_opts(mode=mode, tol=1e-8, n_iter=400, kinetic_balance=1, batch_graph=graph)
            Xs = blocks()
            torch.cuda.synchronize()
            t = time.perf_counter()
            lams, _, infos, _ = dk.lobpcgf_solve_batch(bb, list(range(len(systems))), ns, Xs, o,
                                                       item_buffer=bufs)
            torch.cuda.synchronize()
            batch[f"{tag}_batch_s"] = time.perf_counter() - t
            if graph:
                ex = {}
                for i_ in infos:
                    ex[str(i_["graph_exit"])] = ex.get(str(i_["graph_exit"]), 0) + 1
                batch[f"{tag}_graph_exits"] = ex
                batch[f"{tag}_graph_iterations"] = sum(i_["graph_iterations"] for i_ in infos)
            batch[f"{tag}_batch_converged"] = sum(int(i_["converged"]) for i_ in infos)
            batch[f"{tag}_batch_worst_resnorm"] = max(i_["max_resnorm"] for i_ in infos)
            batch[f"{tag}_batch_iterations"] = sum(i_["iterations"] for i_ in infos)
            batch[f"{tag}_not_converged"] = [i for i, i_ in enumerate(infos) if not i_["converged"]]
            errs = {str(i): float(np.max(np.abs(lams[i][:wanted[i]] - dense[i][:wanted[i]])))
                    for i in dense}
            batch[f"{tag}_max_abs_err_vs_dense_Ha"] = errs
            batch[f"{tag}_worst_err_vs_dense_Ha"] = max(errs.values()) if errs else None
            log(f"[bench] batch of {len(systems)} uneven systems, {tag}: "
                f"{batch[f'{tag}_batch_s']:.3f}s, {batch[f'{tag}_batch_converged']} converged, "
                f"worst error vs dense {batch[f'{tag}_worst_err_vs_dense_Ha']}")
        Xs = blocks()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(len(systems)):
            o = dk.default_opts(mode=dk.MODE_FP64, tol=1e-8, n_iter=400, kinetic_balance=1,
                                n_buffer=bufs[i])
            dk.lobpcgf_solve(bb, i, ns[i], Xs[i], o)
        torch.cuda.synchronize()
        batch["fp64_sequential_s"] = time.perf_counter() - t
        log(f"[bench] same systems one after another, fp64: {batch['fp64_sequential_s']:.3f}s")
        bb.close()

    layered = run_layered() if not args.no_solve and not args.no_batch else None

    # ---- CPU oracle on a bounded sample: one Algorithm 1 iteration on the same system
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import dks as odks, lobpcgf as olob
        op = odks.DKSOperator(s)
        phio = sysgen.start_block(op.miller, s.lattice, s.kpts[0], n, 0)
        X0o = olob.kinetic_balance(op, phio)
        X0o = X0o.reshape(n, -1).T
        C, Om = olob.filter_constants(op.spectrum_bounds(), s.c)
        ah = olob.block_apply(op)

        def pc(R):   # the preconditioner the library applies by default
            return olob.dirac_teter(R, op.q, s.c)

        t = time.perf_counter()
        olob.lobpcgf(ah, X0o, n, C, Om, n_init=0, n_iter=0, tol=1e-300, precond=pc)
        t_init = time.perf_counter() - t
        t = time.perf_counter()
        olob.lobpcgf(ah, X0o, n, C, Om, n_init=0, n_iter=1, tol=1e-300, precond=pc)
        t_one = time.perf_counter() - t
        it_s = max(t_one - t_init, 1e-9)
        from oracle.dks import _WORKERS
        cpu = {"value": 1.0 / it_s, "unit": "iterations/s", "cores": _WORKERS, "kind": "oracle",
               "sample": "one FP64 Algorithm 1 iteration (Teter preconditioner + filter + H.Y + "
                         "Gram + eigh + updates, "
                         "40 bands) on the same heavy-dimer system, timed as t(1 iteration) - "
                         "t(0 iterations) of the numpy/scipy oracle",
               "seconds_per_iteration": it_s}
        log(f"[bench] CPU oracle: {it_s:.2f} s / iteration on {_WORKERS} threads")

    out = {
        "metric": "LOBPCG-F iters/s and H·X spinor-bands/s; FP32-mixed vs FP64 at 1e-8 Ha",
        "value": 1000.0 / step_ms,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "heavy_dimer: cubic 20 bohr, Gamma, Ecut 30 Ha, N_pw 62669 x 4, "
                               "96^3 grid, c 137.036, 40 bands, l<=2 SOC projectors, seeds 0-2 "
                               "(median)",
                   "bands": n, "npw": N, "grid": list(grid), "precision": "fp64",
                   "seeds": [0, 1, 2]},
        "ms_per_step_per_seed": {str(k): v for k, v in per_seed_ms.items()},
        "hx_spinor_bands_per_s": {k: v["spinor_bands_per_s"] for k, v in hx.items()},
        "hx_ms_per_40_bands": {k: v["ms_per_apply"] for k, v in hx.items()},
        "mixed_fp32_iters_per_s": 1000.0 / step32_ms,
        "time_to_solution_1e-8": tts,
        "tiny_dimer": tiny,
        "ksso_comparison": ksso,
        "scf": scf_rec,
        "batch_uneven": batch,
        "layered_kpoints": layered,
        "kernels_apply_H_fp64": kernels,
        "matrix_kernels": mk,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
