#!/usr/bin/env python3
"""Time one probe-position solve of the steam-generator tube model on one GPU.

Workload: the ~2M-tetrahedron tube (conducting tube 9.84/11.11 mm, 1e6 S/m;
support plate 2e6 S/m with four lobed holes; 60 mm air cylinder, 200 mm
long), f = 100 kHz, two coaxial coils at probe position z = 0, plain FP64
GMRES(48) with 64-DOF block-Jacobi (penalty 0.1/mu0 inside the blocks) to
weighted relative residual 1e-8; headline = complex64 inner loop inside the
FP64 outer residual, with the plain FP64 solve timed beside it.

One step = assemble the operator on the device (element kernel, scatter,
equilibration, block inverses), right-hand sides of both coils, the GMRES
solve for the generator coil, V-mean removal and the impedances Z11, Z21.
Mesh topology and the CSR/scatter maps are built once on the host before
timing (they depend on the mesh only).  Inputs are resident in HBM when the
timed region starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or None
    if the kernel source changed since those counters were taken."""
    import hashlib
    try:
        d = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic.json")))
        src = open(os.path.join(ROOT, "paper_1602_03207_amd", "csrc", "kernels.hip"), "rb").read()
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest() != d.get("kernels_hip_sha256"):
        return None
    return d.get("bytes_per_launch", {}).get(kernel)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["tube", "cube"], default="tube")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=48)
    ap.add_argument("--tau-precond-factor", type=float, default=0.1,
                    help="penalty inside the block-Jacobi blocks, as a multiple of tau = 1/mu0")
    ap.add_argument("--max-iter", type=int, default=20000)
    ap.add_argument("--block", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scan", type=int, default=8,
                    help="also time a batched scan of this many probe positions (0 = skip)")
    ap.add_argument("--multifreq", type=int, default=4,
                    help="also time a batch over this many frequencies (100, 240, 400, 600 kHz) x --mf-positions "
                         "probe positions with the frequency-factored matrix, against per-frequency batches (0 = skip)")
    ap.add_argument("--mf-positions", type=int, default=2)
    ap.add_argument("--graph", type=int, default=1,
                    help="also time the headline solve with its Arnoldi chunks as captured HIP graphs (0 = skip)")
    ap.add_argument("--learned-tubes", type=int, default=4,
                    help="perturbed 258k-tet tubes the learned correction trains on (0 = skip)")
    ap.add_argument("--precision", choices=["fp64", "mixed", "mixed16", "all"], default="all",
                    help="headline method; 'all' times mixed16 as the headline and mixed and plain FP64 beside it")
    return ap.parse_args()


def workload(name):
    import numpy as np
    from synth import tube, tube_materials, probe_currents, cube, cube_current
    if name == "tube":
        m = tube()
        nu, sig, omega = tube_materials(1e5)
        J1, J2 = probe_currents(m, 0.0)
        cond = [1, 2, 3]
        tau = float(nu[0])
        desc = {"workload": "sg_tube_2M_tets", "freq_hz": 1e5, "probe_z_m": 0.0}
    else:
        m = cube(8)
        nu, sig, omega = np.array([1.0, 1.0]), np.array([0.0, 1.0]), 50.0
        J1, J2 = cube_current(m, 0), cube_current(m, 1)
        cond = [1]
        tau = 1.0
        desc = {"workload": "unit_cube_n8_3072_tets"}
    return m, nu, sig, omega, J1, J2, cond, tau, desc


def spmv_bytes(M, op, vb=16, gauge=False, nnz_real=0):
    """Algorithmic bytes of one k_spmv launch: values + col + rowptr + x once + y;
    vb = bytes per complex value (16 complex128, 8 complex64); nnz_real
    nonzeros sit in real slices (values of vb / 2 bytes); the gauged variant
    also streams W~ and reads t."""
    n, ne, nv = op.ndof, op.ne, op.nv
    b = (vb + 4) * M.nnz - (vb // 2) * nnz_real + 4 * (n + 1) + 2 * vb * n
    if gauge:
        b += 12 * M.nnz_w + 4 * (ne + 1) + 16 * nv
    return b


def wt_bytes(M, op):
    return 12 * M.nnz_w + 4 * (op.nv + 1) + 16 * op.ne + 16 * op.nv + 8 * op.nv


def block_apply_bytes(M, op, block, vb=16, mb=None):
    """Block inverses (mb bytes per complex entry) + block pointers + DOF list + r gather
    + z scatter (vb bytes per complex vector entry)."""
    import numpy as np
    ptr, _ = M.blocks(block)
    sz = np.diff(ptr).astype(np.int64)
    mb = vb if mb is None else mb
    return int(mb * (sz * sz).sum() + 4 * (len(ptr)) + 4 * op.ndof + 2 * vb * op.ndof)


def learned_section(args, op, b, head):
    """Train the learned coarse correction on perturbed tubes (solver-generated
    pairs, GPU training kernels), then solve the headline right-hand side with
    it; untimed by the headline, reported beside it."""
    import numpy as np
    import torch
    from synth import perturbed_tube, tube_materials, probe_currents
    from paper_1602_03207_amd import eddy, learned
    kw = dict(h_z=1e-3, h_z_end=20e-3, h_theta=2e-3, n_theta_max=48, h_wall=0.4e-3, h_coil=1.0e-3, h_core=2e-3,
              h_out=6e-3)
    t0 = time.perf_counter()
    sets, keep, nt = [], [], 0
    for seed in range(args.learned_tubes):
        m, (ft, fp) = perturbed_tube(seed, **kw)
        nu, sig, omega = tube_materials(1e5, sigma_tube=1e6 * ft, sigma_plate=2e6 * fp)
        M = eddy.Mesh(m.xyz, m.tet, m.region, [0, 1, 1, 1])
        o = eddy.Operator(M, tau=float(nu[0]), block_size=args.block, tau_precond=args.tau_precond_factor * nu[0])
        o.assemble(nu, sig, omega)
        B = [o.rhs_from_current(torch.from_numpy(np.ascontiguousarray(probe_currents(m, z)[0])).cuda())
             for z in (-12e-3, 0.0, 12e-3)]
        X, C, W = learned.collect_pairs(o, B, restart=args.restart, precision=head)
        sets.append((o, X, C, W))
        keep.append(M)
        nt = m.nt
    zero = torch.zeros(eddy.GNN_PARAMS, dtype=torch.float32, device="cuda")
    l0 = float(np.mean([learned.mean_loss(o, zero, X, C, W) for o, X, C, W in sets]))
    theta, _ = learned.train(sets, steps=400, batch=32, lr=2e-3, log_every=0)
    l1 = float(np.mean([learned.mean_loss(o, theta, X, C, W) for o, X, C, W in sets]))
    t_train = time.perf_counter() - t0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    xp, rp = op.solve(b[0], tol=args.tol, restart=args.restart, max_iter=args.max_iter, precision=head)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    xl, rl = op.solve(b[0], tol=args.tol, restart=args.restart, max_iter=args.max_iter, precision=head,
                      gnn_theta=theta)
    torch.cuda.synchronize()
    tl = time.perf_counter() - t2
    tp = t2 - t1
    diff = float((torch.linalg.norm(xl - xp) / torch.linalg.norm(xp)).item())
    return {"train": {"tubes": args.learned_tubes, "tets_each": nt, "pairs": int(sum(X.shape[0] for _, X, _, _ in sets)),
                      "loss_c0": round(l0, 5), "loss_trained": round(l1, 5), "seconds": round(t_train, 1)},
            "solve_s": round(tl, 4), "iters": rl.iters, "learned_cycles": rl.learned_cycles,
            "fell_back": rl.fell_back, "converged": rl.converged, "relres": rl.relres,
            "plain_solve_s": round(tp, 4), "plain_iters": rp.iters,
            "speedup_vs_plain": round(tp / tl, 3), "rel_diff_vs_plain": diff}


def cpu_baseline(args, gpu_iters):
    """The oracle, timed on a bounded sample of the same workload.

    Sample: the tube cross-section over a shortened axis (same radial and
    azimuthal mesh, same conductors and coils, z in [-2, 2] mm with the
    scan-zone spacing), full oracle setup (assembly, equilibration, dense
    block inverses) plus one GMRES(30) cycle.  Scaled to the full workload as
    setup * (nt_full / nt_sample) + (per-iteration time) * (ndof_full /
    ndof_sample) * (GPU iteration count).
    """
    import numpy as np
    from synth import tube, tube_materials, probe_currents
    from oracle.assemble import assemble
    from oracle.solve import BlockJacobi, gmres, equilibration
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = 1
    m = tube(scan_half=2e-3, z_half=2e-3, plate_half=1.6e-3)
    nu, sig, omega = tube_materials(1e5)
    J1, _ = probe_currents(m, 0.0)
    t0 = time.perf_counter()
    s = assemble(m.xyz, m.tet, m.region, nu, sig, omega, tau=nu[0], conductor_regions=[1, 2, 3])
    b = s.rhs(J1)
    sc = equilibration(s)
    P = BlockJacobi.build(s, m.xyz, args.block, scale=sc)
    t1 = time.perf_counter()
    k = args.restart
    res = gmres(lambda v: sc * s.matvec(sc * v), sc * b, P.apply, m=k, tol=1e-30, max_iter=k)
    t2 = time.perf_counter()
    return m.nt, s.ndof, t1 - t0, (t2 - t1) / max(res.iters, 1), threads


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): right-hand sides shard across GPUs "
              f"without communication, but no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1602_03207_amd import eddy

    m, nu, sig, omega, J1, J2, cond, tau, desc = workload(args.workload)
    flags = np.zeros(len(nu), np.int32)
    flags[cond] = 1
    th0 = time.perf_counter()
    M = eddy.Mesh(m.xyz, m.tet, m.region, flags)
    op = eddy.Operator(M, tau=tau, block_size=args.block, tau_precond=tau * args.tau_precond_factor)
    torch.cuda.synchronize()
    host_setup = time.perf_counter() - th0
    J1d = torch.from_numpy(np.ascontiguousarray(J1)).cuda()
    J2d = torch.from_numpy(np.ascontiguousarray(J2)).cuda()
    b = torch.empty((2, op.ndof), dtype=torch.complex128, device="cuda")
    x = torch.empty(op.ndof, dtype=torch.complex128, device="cuda")

    def make_step(prec, graph=False):
        def step():
            op.assemble(nu, sig, omega)
            op.rhs_from_current(J1d, out=b[0])
            op.rhs_from_current(J2d, out=b[1])
            _, rep = op.solve(b[0], tol=args.tol, restart=args.restart, max_iter=args.max_iter, out=x,
                              precision=prec, graph=graph)
            Z = op.impedance(x[None], b, [1.0, 1.0])
            return rep, Z
        return step

    def timed(prec, graph=False):
        step = make_step(prec, graph)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        op.profile(True)
        t0 = time.perf_counter()
        reps = []
        for _ in range(args.steps):
            reps.append(step())
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        prof = op.profile(False)
        vb = 8 if prec in ("mixed", "mixed16") else 16
        mb = 4 if prec == "mixed16" else vb
        kb = {"block_apply": block_apply_bytes(M, op, args.block, vb, mb), "gauge_wt": wt_bytes(M, op),
              "spmv": spmv_bytes(M, op, vb, gauge=reps[-1][0].gauge_in_operator,
                                 nnz_real=op.tuning()["sell_nnz_real"])}
        kernels = {}
        for name, (ms, cnt) in prof.items():
            avg = ms / max(cnt, 1)
            entry = {"avg_ms": round(avg, 5), "launches": cnt, "total_ms": round(ms, 2)}
            if name in kb and cnt:
                gbs = kb[name] / (avg * 1e-3) / 1e9
                entry.update({"bytes_per_launch": kb[name], "GB/s": round(gbs, 1),
                              "frac": round(gbs / HBM_PEAK_GBS, 4)})
            kernels[name] = entry
        rep, Z = reps[-1]
        return {"sec": elapsed / args.steps, "rep": rep, "Z": Z, "kernels": kernels}

    head = "mixed16" if args.precision == "all" else args.precision
    runs = {head: timed(head)}
    graph_run = timed(head, graph=True) if args.graph else None
    if args.precision == "all":
        runs["mixed"] = timed("mixed")
        runs["fp64"] = timed("fp64")
    H = runs[head]
    rep, Z, kernels = H["rep"], H["Z"], H["kernels"]
    sec_per_solve = H["sec"]
    knames = {"block_apply": "k_block_apply", "gauge_wt": "k_wt", "spmv": "k_spmv_sell"}
    ktypes = {"fp64": "<double2>", "mixed": "<float2>", "mixed16": "<float2>"}
    single = {k: v for k, v in kernels.items() if k in knames and v["launches"]}
    roof = None
    if single:
        dom = max(single, key=lambda k: single[k]["total_ms"])
        d = single[dom]
        kname = knames[dom] + ktypes[head]
        if dom == "block_apply":      # storage of the vector, the inverses, the input
            kname = {"fp64": "k_block_apply<double2, double2, double2>",
                     "mixed": "k_block_apply<float2, float2, float2>",
                     "mixed16": "k_block_apply<float2, unsigned int, hbasis>"}[head]
        roof = {"bound": "hbm", "kernel": kname, "achieved": d["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["frac"], "traffic": measured_traffic(kname),
                "algorithmic_bytes": d["bytes_per_launch"]}

    scan = None
    if args.scan and args.workload == "tube":
        from synth import probe_currents
        zs = np.linspace(-20e-3, 20e-3, args.scan)
        Js = [torch.from_numpy(np.ascontiguousarray(probe_currents(m, float(z))[0])).cuda() for z in zs]
        J2s = [torch.from_numpy(np.ascontiguousarray(probe_currents(m, float(z))[1])).cuda() for z in zs]
        Bs = torch.empty((args.scan, op.ndof), dtype=torch.complex128, device="cuda")
        B2s = torch.empty_like(Bs)
        Xs = torch.empty_like(Bs)

        def scan_step():
            op.assemble(nu, sig, omega)
            for k in range(args.scan):
                op.rhs_from_current(Js[k], out=Bs[k])
                op.rhs_from_current(J2s[k], out=B2s[k])
            _, reps = op.solve_batched(Bs, tol=args.tol, restart=args.restart, max_iter=args.max_iter, out=Xs,
                                       precision=head)
            Zs = [op.impedance(Xs[k:k + 1], torch.stack([Bs[k], B2s[k]]), [1.0, 1.0]) for k in range(args.scan)]
            return reps, Zs

        scan_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sreps, sZ = scan_step()
        torch.cuda.synchronize()
        st = time.perf_counter() - t0
        scan = {"positions": args.scan, "z_mm": [round(float(z) * 1e3, 3) for z in zs],
                "s_per_position": round(st / args.scan, 4), "s_per_scan": round(st, 3),
                "iters": [r.iters for r in sreps], "converged": all(r.converged for r in sreps),
                "max_relres": max(r.relres for r in sreps),
                "speedup_vs_single_headline": round(sec_per_solve / (st / args.scan), 3),
                "Z11": [[z[0, 0].real, z[0, 0].imag] for z in sZ]}

    mfreq = None
    if args.multifreq and args.workload == "tube":
        from synth import probe_currents, tube_materials
        freqs = [1e5, 2.4e5, 4e5, 6e5][:args.multifreq]
        ops_f = []
        for f in freqs:
            o2 = op if f == 1e5 else eddy.Operator(M, tau=tau, block_size=args.block,
                                                   tau_precond=tau * args.tau_precond_factor)
            o2.assemble(nu, sig, tube_materials(f)[2])
            ops_f.append(o2)
        zs = np.linspace(-2e-3, 2e-3, args.mf_positions)
        P = len(zs)
        Bm = torch.stack([ops_f[0].rhs_from_current(torch.from_numpy(np.ascontiguousarray(
            probe_currents(m, float(z))[0])).cuda()) for _ in freqs for z in zs])
        idx = [fi for fi in range(len(freqs)) for _ in zs]
        kw = dict(tol=args.tol, restart=args.restart, max_iter=args.max_iter, precision=head)
        eddy.solve_multifreq(ops_f, Bm, idx, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Xm, mreps = eddy.solve_multifreq(ops_f, Bm, idx, **kw)
        torch.cuda.synchronize()
        t_mf = time.perf_counter() - t0
        t0 = time.perf_counter()
        sreps_f = []
        for fi, o2 in enumerate(ops_f):
            _, r2 = o2.solve_batched(Bm[fi * P:(fi + 1) * P].clone(), **kw)
            sreps_f += r2
        torch.cuda.synchronize()
        t_sep = time.perf_counter() - t0
        mfreq = {"freqs_hz": freqs, "positions_per_freq": P, "systems": len(idx),
                 "s_per_system": round(t_mf / len(idx), 4), "s_per_system_per_frequency_batches": round(t_sep / len(idx), 4),
                 "speedup_vs_per_frequency_batches": round(t_sep / t_mf, 3),
                 "iters": [r.iters for r in mreps], "iters_per_frequency_batches": [r.iters for r in sreps_f],
                 "converged": all(r.converged for r in mreps) and all(r.converged for r in sreps_f),
                 "max_relres": max(r.relres for r in mreps)}
        del ops_f, Xm, Bm

    learned_out = None
    if args.learned_tubes and args.workload == "tube":
        learned_out = learned_section(args, op, b, head)

    cpu = None
    if not args.no_cpu_baseline and args.workload == "tube":
        it_cpu = runs["fp64"]["rep"].iters if "fp64" in runs else rep.iters
        nt_s, nd_s, t_setup, t_it, threads = cpu_baseline(args, it_cpu)
        est = t_setup * (M.nt / nt_s) + t_it * (op.ndof / nd_s) * it_cpu
        cpu = {"value": round(est, 2), "unit": "s per probe-position solve", "cores": threads, "kind": "oracle",
               "sample": (f"oracle on the tube cross-section over z in [-2,2] mm ({nt_s} tets, {nd_s} DOF): "
                          f"setup {t_setup:.2f} s + {t_it:.3f} s per GMRES iteration, scaled linearly to "
                          f"{M.nt} tets / {op.ndof} DOF and to the GPU's {it_cpu} plain-FP64 iterations")}

    out = {
        "metric": "s per probe-position solve at rel-res 1e-8 (learned/mixed vs plain FP64); SpMV GB/s",
        "value": round(sec_per_solve, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec_per_solve * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "c64 inner / c128 outer", "mixed16": "c64 inner, c16 block inverses / c128 outer",
                  "fp64": "c128 (f64)"}[head],
        "data": "synthetic",
        "config": {**desc, "tets": M.nt, "dof": op.ndof, "nnz": M.nnz, "nnz_w": M.nnz_w, "block": args.block,
                   "restart": args.restart, "tol": args.tol, "precision": head, "parallelism": "single GPU",
                   "tau_precond_factor": args.tau_precond_factor},
        "solve": {"iters": rep.iters, "restarts": rep.restarts, "converged": rep.converged, "relres": rep.relres,
                  "projection_cg_iters": rep.cg_iters,
                  "Z11": [Z[0, 0].real, Z[0, 0].imag], "Z21": [Z[0, 1].real, Z[0, 1].imag]},
        "mixed_c64_inverses": ({"s_per_solve": round(runs["mixed"]["sec"], 4), "iters": runs["mixed"]["rep"].iters,
                                "converged": runs["mixed"]["rep"].converged, "relres": runs["mixed"]["rep"].relres,
                                "speedup_of_headline": round(runs["mixed"]["sec"] / sec_per_solve, 3),
                                "Z11": [runs["mixed"]["Z"][0, 0].real, runs["mixed"]["Z"][0, 0].imag]}
                               if "mixed" in runs and head != "mixed" else None),
        "plain_fp64": ({"s_per_solve": round(runs["fp64"]["sec"], 4), "iters": runs["fp64"]["rep"].iters,
                        "converged": runs["fp64"]["rep"].converged, "relres": runs["fp64"]["rep"].relres,
                        "speedup_of_headline": round(runs["fp64"]["sec"] / sec_per_solve, 3),
                        "Z11": [runs["fp64"]["Z"][0, 0].real, runs["fp64"]["Z"][0, 0].imag],
                        "kernels": runs["fp64"]["kernels"]} if "fp64" in runs and head != "fp64" else None),
        "graph": ({"s_per_solve": round(graph_run["sec"], 4), "iters": graph_run["rep"].iters,
                   "speedup_vs_eager": round(sec_per_solve / graph_run["sec"], 3),
                   "same_iterations": graph_run["rep"].iters == rep.iters} if graph_run else None),
        "batched_scan": scan,
        "multifreq_batch": mfreq,
        "learned": learned_out,
        "host_setup_s": round(host_setup, 2),
        "spmv_tuning": op.tuning(),
        "kernels": kernels,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
