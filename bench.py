#!/usr/bin/env python3
"""Benchmark: one Newton-step linear solve of the condensed ALE FSI system.

A step is the whole hot path on one batch of synthetic input resident in HBM:
  momentum solve (FGMRES + V-cycle + additive Vanka, eq. problem:1)
  -> condensed deformation update du = k theta dv on interface/solid nodes
  -> deformation system M du = M (k theta dv) solved by the same machinery
  -> ALE extension solve E_f du_f = b5 - E_i du_i (eq. problem:3).
Workload (default): 3D box [0,1]^3, solid block [0.3,0.7]x[0.4,0.6]^2, 32^3 Q2
hexes (65^3 nodes), 4 levels, rel. residual 1e-8 (FP64-checked).

Prints ONE JSON line (rank 0).  value = (momentum + ALE unknowns) solved per
second of step wall time, FP64 path; the FP32-mixed path is reported in the
same line under "mixed".
"""
import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix rate
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector rate


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def vanka_bytes(npatch, np_, nl, s):
    """Algorithmic bytes of one Vanka patch-kernel launch: every patch streams
    its n_p x n_p inverse once, gathers n_p residual entries, writes n_p
    corrections and reads its node list."""
    return npatch * (np_ * np_ * s + 2 * np_ * s + nl * 4)


def spmv_bytes(nnzb, nrows, b, s):
    """Algorithmic bytes of one residual SpMV d = r - A x: block values and
    column indices once, row pointers, x, r and d once, the mask bytes."""
    return nnzb * (b * b * s + 4) + 4 * (nrows + 1) + 3 * nrows * b * s + nrows * b


KERNEL_SOURCES = ("batch_kernels.hip", "device_ops.h")
ASM_SOURCES = ("kernels_asm.hip",)
# the batched kernels (and their helpers) whose source keys each role's counter entry
ROLE_KERNEL = {"vanka_patch": ("kb_vanka_patch",), "spmv_residual": ("kb_spmv",),
               "restrict": ("kb_restrict", "taps_1d", "kb_restrict3"), "prolong": ("kb_prolong", "prolong_node4")}


def _function_text(src, name):
    """the text of the first definition of `name` (up to its closing brace)"""
    import re
    m = re.search(r"\b" + re.escape(name) + r"\s*\(", src)
    if not m:
        return ""
    i = src.index("{", m.end())
    depth = 0
    for j in range(i, len(src)):
        depth += {"{": 1, "}": -1}.get(src[j], 0)
        if depth == 0:
            return src[m.start():j + 1]
    return src[m.start():]


def kernel_source_hash(sources=KERNEL_SOURCES, role=None):
    """sha256[:16] over the sources that define the kernels measured: for a
    batched-kernel role, the device functions (device_ops.h) and that
    kernel's own definition; otherwise the whole files."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1904_02401_amd", "csrc")
    if role in ROLE_KERNEL:
        h.update(open(os.path.join(csrc, "device_ops.h"), "rb").read())
        src = open(os.path.join(csrc, "batch_kernels.hip")).read()
        for name in ROLE_KERNEL[role]:
            h.update(_function_text(src, name).encode())
        return h.hexdigest()[:16]
    for f in sources:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(role, workload, prec, sources=KERNEL_SOURCES):
    """HBM bytes per launch recorded from rocprofv3 counters, or None when the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    cur = kernel_source_hash(sources, role if sources == KERNEL_SOURCES else None)
    for line in open(path):
        f = line.split()
        if len(f) == 5 and not line.startswith("#") and f[:3] == [role, workload, prec]:
            return float(f[3]) if f[4] == cur else None
    return None


def _split_err(x, ref, b):
    """relative 2-norm error of the velocity and of the pressure components
    (their scales differ by orders of magnitude)."""
    import numpy as np
    x, ref = x.reshape(-1, b), ref.reshape(-1, b)
    out = {}
    for name, sl in (("velocity", slice(1, b)), ("pressure", slice(0, 1))):
        out[name] = float(np.linalg.norm(x[:, sl] - ref[:, sl]) / max(np.linalg.norm(ref[:, sl]), 1e-300))
    return out


def kernels_only(P, precision, reps):
    """Launch only the finest-level smoother step (residual SpMV + Vanka patch
    kernel + gather) of the momentum system `reps` times: the workload of the
    hardware-counter runs."""
    import torch
    from paper_1904_02401_amd import fsimg
    from paper_1904_02401_amd.problems import level_dicts
    ctx = fsimg.fsimg_ctx_create(0)
    h = fsimg.fsimg_hier_create(ctx, level_dicts(P, "mom"), fsimg.fsimg_default_opts(precision=precision))
    fsimg.fsimg_factor(h)
    dt = torch.float64 if precision == fsimg.FSIMG_FP64 else torch.float32
    b = torch.tensor(P.rhs["mom"], device="cuda:0", dtype=dt)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    for _ in range(reps):
        fsimg.fsimg_vanka_step(h, 0, precision, b, x)
    torch.cuda.synchronize()
    fsimg.fsimg_hier_destroy(h)
    fsimg.fsimg_ctx_destroy(ctx)
    log(f"kernels-only: {reps} finest-level smoothing steps done")


def calib_copy(nbytes, reps):
    """Plain device-to-device copy of a known size (counter calibration)."""
    import torch
    a = torch.empty(nbytes // 8, device="cuda:0", dtype=torch.float64).fill_(1.0)
    c = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        c.copy_(a)
    torch.cuda.synchronize()
    log(f"calib-copy: {reps} copies of {nbytes} bytes")


def run_gpu(P, precision, steps, warmup, with_mass=True, tune=True, patches=0, schedule=0, smoother=0,
            lookahead=2, small_kib=0, omega=0.8):
    import torch
    from paper_1904_02401_amd import fsimg
    from paper_1904_02401_amd.problems import level_dicts

    dev = torch.device("cuda:0")
    ctx = fsimg.fsimg_ctx_create(0)
    hs = {}
    t0 = time.perf_counter()
    systems = ["mom", "ale"] + (["mass"] if with_mass else [])
    sched_ms = {}
    for name in systems:
        o = fsimg.fsimg_default_opts(precision=precision, profile=0, vanka_patches=patches,
                                     vanka_schedule=max(schedule, 0), smoother=smoother,
                                     krylov_lookahead=lookahead, small_level_kib=small_kib, omega=omega)
        if schedule < 0:  # auto: the fastest schedule, measured on this system's hierarchy
            ms, best = fsimg.fsimg_tune_schedule(ctx, level_dicts(P, name), o, reps=3)
            sched_ms[name] = {"gather": ms[0], "parity": ms[1], "greedy": ms[2], "chosen": best}
            o.vanka_schedule = best
        hs[name] = fsimg.fsimg_hier_create(ctx, level_dicts(P, name), o)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    for name in systems:
        fsimg.fsimg_factor(hs[name])
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0
    t0 = time.perf_counter()
    shapes = {}
    if tune:
        # launch shapes measured on these hierarchies (no result bit depends on them)
        for name in systems:
            fsimg.fsimg_hier_tune(hs[name])
        torch.cuda.synchronize()
        word = 8 if precision == fsimg.FSIMG_FP64 else 4
        for name in systems:
            for l in range(len(P.levels) - 1):
                info = fsimg.fsimg_hier_info(hs[name], l)
                m = P.levels[l].systems[name]
                shapes[f"{name}/L{l}"] = {
                    "spmv_rows_per_wave": fsimg.fsimg_tune_get(ctx, fsimg.FSIMG_TUNE_SPMV_ROWS, m.b, word,
                                                               m.nrows),
                    "vanka_patches_per_wg": fsimg.fsimg_tune_get(ctx, fsimg.FSIMG_TUNE_VANKA_PPW,
                                                                 info["np"], word, max(info["npatch"], 1))}
    t_tune = time.perf_counter() - t0
    lev = P.levels[0]
    nn = lev.nnodes
    d = P.dim
    k, th = P.params["k"], P.params["theta"]
    b_mom = torch.tensor(P.rhs["mom"], device=dev)
    b_ale = torch.tensor(P.rhs["ale"], device=dev)
    node_mask = torch.tensor(lev.node_solid, device=dev)
    x_mom = torch.zeros_like(b_mom)
    x_ale = torch.zeros(nn * d, device=dev, dtype=torch.float64)
    b_mass = torch.zeros_like(x_ale)
    x_mass = torch.zeros_like(x_ale)
    stream = torch.cuda.current_stream()

    def step(profile=False):
        x_mom.zero_()
        if profile:
            opts_prof(hs["mom"], 1)
        st_m = fsimg.fsimg_solve(hs["mom"], b_mom, x_mom, stream, raise_on_noconv=False)
        if profile:
            opts_prof(hs["mom"], 0)
        fsimg.fsimg_deform_update(nn, d, node_mask, k, th, x_mom, d + 1, 1, None, None, x_ale, stream)
        st_s = None
        if with_mass:
            fsimg.fsimg_level_apply(hs["mass"], 0, fsimg.FSIMG_FP64, x_ale, b_mass, stream)
            x_mass.zero_()
            st_s = fsimg.fsimg_solve(hs["mass"], b_mass, x_mass, stream, raise_on_noconv=False)
        st_a = fsimg.fsimg_solve(hs["ale"], b_ale, x_ale, stream, raise_on_noconv=False)
        return st_m, st_s, st_a

    def opts_prof(h, on):
        fsimg.fsimg_hier_set_profile(h, on)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, lat = [], []
    for _ in range(steps):
        ts = time.perf_counter()
        stats.append(step())  # every solve returns to the host when it has converged
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps
    # per-kernel timing with HIP events on the launch stream, over one more
    # set of timed steps (the same work)
    prof = [step(profile=True)[0] for _ in range(max(1, min(steps, 3)))]
    torch.cuda.synchronize()
    # the finest momentum level's patch factorisation (MFMA), event-timed on
    # the launch stream; refactoring the same values reproduces the inverses
    opts_prof(hs["mom"], 1)
    factor_ms = []
    for _ in range(3):
        fsimg.fsimg_factor(hs["mom"], stream)
        factor_ms.append(fsimg.fsimg_hier_info(hs["mom"], 0)["factor_ms"])
    opts_prof(hs["mom"], 0)
    info_m = fsimg.fsimg_hier_info(hs["mom"], 0)
    res = dict(t_step=t_step, t_setup=t_setup, t_factor=t_factor, t_tune=t_tune, shapes=shapes,
               schedule_ms=sched_ms,
               stats=stats[-1], prof=prof, factor_ms=factor_ms, lat=lat,
               solve_ms={k: [st[j]["solve_ms"] for st in stats if st[j] is not None]
                         for j, k in enumerate(("mom", "mass", "ale"))},
               info_m=info_m, x_mom=x_mom.cpu().numpy(), x_ale=x_ale.cpu().numpy())
    for h in hs.values():
        fsimg.fsimg_hier_destroy(h)
    fsimg.fsimg_ctx_destroy(ctx)
    return res


def asm_flops_per_element(dim, solid):
    """Algorithmic flops of one element Jacobian as the kernel's formula
    states it: per (row node, column node, Gauss point) the fluid block
    (inertia, transport, convection, viscous, pressure, divergence and
    stabilisation entries) costs 100 flops in 3D / 57 in 2D, the solid block
    (mass and the linearised first Piola stress) 129 / 62; 3^d Gauss points,
    (3^d)^2 node pairs."""
    nn = 3 ** dim
    per = (129 if solid else 100) if dim == 3 else (62 if solid else 57)
    return nn * nn * nn * per


def asm_roofline(f, P, x, u, xo, uo, workload):
    """The finest level's element kernels, event-timed per launch on the
    launch stream (three Jacobian and residual assemblies at the given
    state): the Jacobian kernel's roofline entry, the residual kernel's
    launch time and the finest level's assembly rate (elements / s)."""
    import torch
    from paper_1904_02401_amd import fsimg
    fsimg.fsimg_fsi_set_profile(f, 1)
    for _ in range(3):
        fsimg.fsimg_fsi_jacobian(f, x, u, xo, uo)
        res = torch.empty_like(x)
        fsimg.fsimg_fsi_residual(f, x, u, xo, uo, res)
    prof = fsimg.fsimg_fsi_profile(f)
    fsimg.fsimg_fsi_set_profile(f, 0)
    lev = P.levels[0]
    ns = int(lev.cell_solid.sum())
    nf = lev.ncells - ns
    flops = nf * asm_flops_per_element(P.dim, False) + ns * asm_flops_per_element(P.dim, True)
    launches_per_pass = 2 ** P.dim
    jac_pass_ms = prof["jac_ms"] / max(prof["jac_launches"], 1) * launches_per_pass
    avg_launch_ms = prof["jac_ms"] / max(prof["jac_launches"], 1)
    tf = flops / (jac_pass_ms * 1e-3) / 1e12
    nb = lev.systems["mom"].nnzb
    b = P.dim + 1
    # bytes the colouring moves: every element reads and writes its (3^d)^2 blocks
    rmw_bytes = lev.ncells * (3 ** P.dim) ** 2 * b * b * 8 * 2
    roof = {"bound": "alu", "kernel": f"k_asm_jac<{P.dim}>", "achieved": tf,
            "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": measured_traffic("asm_jac", workload, "fp64", ASM_SOURCES),
            "rmw_bytes_per_launch": rmw_bytes / launches_per_pass,
            "flops_per_launch": flops / launches_per_pass, "avg_launch_ms": avg_launch_ms,
            "launches": prof["jac_launches"],
            "rmw_GBs": rmw_bytes / (jac_pass_ms * 1e-3) / 1e9,
            "matrix_bytes": nb * b * b * 8}
    res_kernel = {"kernel": f"k_asm_res<{P.dim}>",
                  "avg_launch_ms": prof["res_ms"] / max(prof["res_launches"], 1),
                  "launches": prof["res_launches"]}
    return roof, res_kernel, lev.ncells / (jac_pass_ms * 1e-3)


# (dimension, levels, curved): the rectilinear channel (square prism) and the
# curved one (isoparametric Q2 cells: the cylinder, rows of even height away
# from obstacle and beam)
CHANNEL_CONFIGS = {"channel3": (3, 4, False), "channel2": (2, 5, False),
                   "channel3c": (3, 4, True), "channel2c": (2, 5, True)}


def run_channel(args):
    """The benchmark channel of Sec. 5 from rest: time steps of the start-up
    (inflow ramped by (1 - cos(pi t)) / 2), each one fsimg_fsi_time_step
    (old level <- state, inflow rows, Newton loop with Jacobian reuse) and
    one fsimg_fsi_force (drag and lift in residual form)."""
    import numpy as np
    import torch
    from fsigen import inflow_ramp, make_channel
    from paper_1904_02401_amd import fsimg
    from paper_1904_02401_amd.problems import fsi_levels, level_dicts

    dim, nlev, curved = CHANNEL_CONFIGS[args.config]
    t0 = time.perf_counter()
    C = make_channel(dim, nlev, curved=curved)
    P = C.problem
    lev = P.levels[0]
    log(f"{args.config}: {lev.cells} cells on the finest of {nlev} levels, generated in "
        f"{time.perf_counter() - t0:.1f} s")
    prec = fsimg.FSIMG_FP64 if args.only == "fp64" else fsimg.FSIMG_MIXED
    tag = "fp64" if prec == fsimg.FSIMG_FP64 else "mixed"
    ctx = fsimg.fsimg_ctx_create(0)
    # the channel's cells reach aspect ratio 24 (the beam's rows run the whole
    # length): element patches stall there, block patches (2^d elements) do not
    patches = args.patches or "block"
    o = fsimg.fsimg_default_opts(precision=prec, max_iter=1000, vanka_patches=(
        fsimg.FSIMG_PATCH_BLOCK if patches == "block" else fsimg.FSIMG_PATCH_ELEMENT))
    t0 = time.perf_counter()
    mom = fsimg.fsimg_hier_create(ctx, level_dicts(P, "mom"), o)
    ale = fsimg.fsimg_hier_create(ctx, level_dicts(P, "ale"), o)
    f = fsimg.fsimg_fsi_create(mom, ale, fsi_levels(P), P.params)
    if not args.no_tune:
        fsimg.fsimg_factor(mom)
        fsimg.fsimg_factor(ale)
        fsimg.fsimg_hier_tune(mom)
        fsimg.fsimg_hier_tune(ale)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    n, d = lev.nnodes, dim
    x = torch.zeros(n * (d + 1), device=dev, dtype=torch.float64)
    u = torch.zeros(n * d, device=dev, dtype=torch.float64)
    xo, uo = x.clone(), u.clone()
    rows = torch.tensor(C.inflow_rows, device=dev)
    vals = torch.tensor(C.inflow_vals, device=dev)
    nodes = torch.tensor(C.force_nodes, device=dev)
    nopts = fsimg.fsimg_default_newton_opts(gamma=args.gamma, lin_rtol=args.lin_rtol, atol=args.newton_atol,
                                            max_steps=args.max_newton, ale_rtol=args.ale_rtol)
    k = P.params["k"]
    hist = []

    def step(i):
        t = i * k
        st = fsimg.fsimg_fsi_time_step(f, x, u, xo, uo, rows, vals, inflow_ramp(t), nopts,
                                       raise_on_noconv=False)
        F = fsimg.fsimg_fsi_force(f, x, u, xo, uo, nodes, d)
        uB = u[C.probe_node * d:(C.probe_node + 1) * d].tolist()   # the beam's probe point
        log(f"t = {t:.4f}: status {st['status']}, {st['steps']} Newton steps, {st['jacobians']} Jacobians, "
            f"res {st['res0']:.3e} -> {st['res']:.3e}, {st['ms_total']:.0f} ms, drag {F[0]:.6e}, "
            f"lift {F[1]:.6e}, u_B {uB[0]:.3e} {uB[1]:.3e}")
        hist.append(dict(t=t, drag=F[0], lift=F[1], u_B=uB, **{q: st[q] for q in (
            "status", "steps", "jacobians", "halvings", "lin_iters_mom", "lin_iters_ale", "ms_total")}))
        return st

    for i in range(1, args.warmup + 1):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step(i) for i in range(args.warmup + 1, args.warmup + args.steps + 1)]
    torch.cuda.synchronize()
    t_ts = (time.perf_counter() - t0) / args.steps
    bad = [h for h in hist if h["status"] != fsimg.FSIMG_OK]
    roof, res_kernel, elems_per_s = asm_roofline(f, P, x, u, xo, uo, f"{args.config}-momentum-level0")
    n_mom = lev.systems["mom"].nrows * lev.systems["mom"].b
    n_ale = lev.systems["ale"].nrows * lev.systems["ale"].b
    tot = lambda q: sum(s[q] for s in stats)
    out = {
        "metric": "benchmark channel time steps: (momentum + ALE unknowns) x time steps per second",
        "value": (n_mom + n_ale) / t_ts,
        "unit": "DoF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_ts * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if tag == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": (f"{args.config}: the {dim}D benchmark channel of Sec. 5 ("
                                + ("the cylinder of radius 0.05 on isoparametric Q2 cells, rows of even "
                                   "height away from obstacle and beam" if curved else
                                   "cylinder read as a square prism")
                                + f"), {'x'.join(map(str, lev.cells))} Q2 cells, {nlev} levels, "
                                f"start-up from rest, time steps {args.warmup + 1}..{args.warmup + args.steps} "
                                f"timed (k = {k}, theta = {P.params['theta']}), each with drag / lift; "
                                f"gamma_nt = {args.gamma}, Newton stop at 1e-8 relative or "
                                f"{args.newton_atol:g} absolute, momentum solves to {args.lin_rtol:g}, "
                                f"ALE solves to {args.ale_rtol or 1e-8:g}, {patches} Vanka patches"),
                   "unknowns_momentum": n_mom, "unknowns_ale": n_ale, "precision": tag,
                   "vanka_patches": patches},
        "roofline": roof,
        "residual_kernel": res_kernel,
        "newton": {"time_steps": args.steps, "newton_steps": tot("steps"), "jacobians": tot("jacobians"),
                   "halvings": tot("halvings"), "momentum_iters": tot("lin_iters_mom"),
                   "ale_iters": tot("lin_iters_ale"), "ms_jacobian_assembly": tot("ms_jacobian") / args.steps,
                   "ms_factor": tot("ms_factor") / args.steps, "ms_solve": tot("ms_solve") / args.steps,
                   "not_converged": len(bad), "setup_s": t_setup},
        "functionals": hist,
        "assembly_elements_per_s": elems_per_s,
    }
    fsimg.fsimg_fsi_destroy(f)
    fsimg.fsimg_hier_destroy(mom)
    fsimg.fsimg_hier_destroy(ale)
    fsimg.fsimg_ctx_destroy(ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_assembly_baseline(P)
    print(json.dumps(out), flush=True)


def run_newton(args, P):
    """Time steps of the approximate Newton loop on the GPU (residual and
    Jacobian assembly, Jacobian reuse, momentum / deformation / ALE solves,
    line search), each from the generator's seeded state."""
    import numpy as np
    import torch
    from paper_1904_02401_amd import fsimg
    from paper_1904_02401_amd.problems import fsi_levels, fsi_state, level_dicts

    prec = fsimg.FSIMG_FP64 if args.only == "fp64" else fsimg.FSIMG_MIXED
    tag = "fp64" if prec == fsimg.FSIMG_FP64 else "mixed"
    ctx = fsimg.fsimg_ctx_create(0)
    o = fsimg.fsimg_default_opts(precision=prec)
    t0 = time.perf_counter()
    mom = fsimg.fsimg_hier_create(ctx, level_dicts(P, "mom"), o)
    ale = fsimg.fsimg_hier_create(ctx, level_dicts(P, "ale"), o)
    f = fsimg.fsimg_fsi_create(mom, ale, fsi_levels(P), P.params)
    if not args.no_tune:
        fsimg.fsimg_factor(mom)
        fsimg.fsimg_factor(ale)
        fsimg.fsimg_hier_tune(mom)
        fsimg.fsimg_hier_tune(ale)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    init = [torch.tensor(a, device=dev) for a in fsi_state(P)]
    x, u, xo, uo = (a.clone() for a in init)
    nopts = fsimg.fsimg_default_newton_opts(gamma=args.gamma, lin_rtol=args.lin_rtol, atol=args.newton_atol,
                                            ale_rtol=args.ale_rtol)

    count = [0]

    def time_step():
        if args.chain and count[0] > 0:
            # t_{n-1} <- the last converged state, which is also the initial guess;
            # the Jacobian is carried over
            xo.copy_(x)
            uo.copy_(u)
        else:
            # one time step from the seeded state, Jacobian assembled afresh: every
            # timed step does the same work
            for dst, src in zip((x, u, xo, uo), init):
                dst.copy_(src)
            fsimg.fsimg_fsi_drop_jacobian(f)
        count[0] += 1
        st = fsimg.fsimg_fsi_newton(f, x, u, xo, uo, nopts, raise_on_noconv=False)
        log(f"newton time step: status {st['status']}, {st['steps']} steps, {st['jacobians']} "
            f"Jacobians, {st['halvings']} halvings, res {st['res0']:.3e} -> {st['res']:.3e}, "
            f"{st['ms_total']:.0f} ms")
        return st

    for _ in range(args.warmup):
        time_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [time_step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_ts = (time.perf_counter() - t0) / args.steps
    for st in stats:
        if st["status"] != fsimg.FSIMG_OK:
            log(f"newton: a time step ended with status {st['status']} after {st['steps']} steps")
    roof, res_kernel, elems_per_s = asm_roofline(f, P, x, u, xo, uo, f"{args.config}-momentum-level0")
    lev = P.levels[0]
    n_mom = lev.systems["mom"].nrows * lev.systems["mom"].b
    n_ale = lev.systems["ale"].nrows * lev.systems["ale"].b
    tot = lambda k: sum(s[k] for s in stats)
    out = {
        "metric": "Newton time steps: (momentum + ALE unknowns) x time steps per second",
        "value": (n_mom + n_ale) / t_ts,
        "unit": "DoF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_ts * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if tag == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": (f"{args.config}: " + (
                       f"{args.warmup + args.steps} successive Newton time steps from the seeded state "
                       f"(the last {args.steps} timed), Jacobian carried over" if args.chain else
                       "one Newton time step from the seeded state, Jacobian assembled afresh") +
                       f" (theta = {P.params['theta']}, k = {P.params['k']}), gamma_nt = {args.gamma}, "
                       f"Newton stop at 1e-8 relative or {args.newton_atol:g} absolute (max-norm), "
                       f"momentum solves to {args.lin_rtol:g} relative, ALE solves to {args.ale_rtol or 1e-8:g}"),
                   "unknowns_momentum": n_mom, "unknowns_ale": n_ale, "precision": tag},
        "roofline": roof,
        "residual_kernel": res_kernel,
        "newton": {"per_step": [{k: st[k] for k in ("status", "steps", "jacobians", "halvings",
                                                    "lin_iters_mom", "lin_iters_ale", "ms_total")}
                                for st in stats],
                   "time_steps": args.steps, "newton_steps": tot("steps"),
                   "jacobians": tot("jacobians"), "halvings": tot("halvings"),
                   "momentum_iters": tot("lin_iters_mom"), "ale_iters": tot("lin_iters_ale"),
                   "ms_residual": tot("ms_residual") / args.steps,
                   "ms_jacobian_assembly": tot("ms_jacobian") / args.steps,
                   "ms_factor": tot("ms_factor") / args.steps, "ms_solve": tot("ms_solve") / args.steps,
                   "res_hist_last": stats[-1]["res_hist"], "setup_s": t_setup},
    }
    fsimg.fsimg_fsi_destroy(f)
    fsimg.fsimg_hier_destroy(mom)
    fsimg.fsimg_hier_destroy(ale)
    fsimg.fsimg_ctx_destroy(ctx)
    # GPU assembly rate of the finest level (elements / s), the oracle's beside it
    out["assembly_elements_per_s"] = elems_per_s
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_assembly_baseline(P)
    print(json.dumps(out), flush=True)


def cpu_assembly_baseline(P, n_elems=1024):
    """The oracle's element assembly on the host: residual and complex-step
    Jacobian over a seeded sample of the finest level's cells, in elements
    per second (the oracle cannot run the whole time step at this size: its
    linear solves are direct)."""
    import numpy as np
    from oracle.fsi import Mesh, element_jacobians, element_subset, operator_value
    from paper_1904_02401_amd.problems import fsi_state
    lev = P.levels[0]
    m = Mesh(lev)
    rng = np.random.default_rng(0)
    sub = element_subset(m, np.sort(rng.choice(lev.ncells, n_elems, replace=False)))
    x, u, xo, uo = fsi_state(P)
    t0, c0 = time.perf_counter(), time.process_time()
    operator_value(sub, P.params, x, u, xo, uo)
    element_jacobians(sub, P.params, x, u, xo, uo)
    dt = time.perf_counter() - t0
    cores = round((time.process_time() - c0) / dt, 1)
    return {"value": n_elems / dt, "unit": "elements/s (residual + Jacobian)", "cores": cores,
            "kind": "oracle",
            "sample": f"residual and complex-step Jacobian of {n_elems} seeded cells of the finest "
                      f"level ({dt:.1f} s); GPU: the same per cell in assembly_elements_per_s"}


def _median_time(fn, reps=3):
    """median wall time of fn() over reps calls"""
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def _oracle_setup(P, name, chunk=(2048, 4096), slab_rows=65536):
    """The untimed inputs of the oracle's sampled operations on system `name`
    (see _oracle_costs): per smoothing level a slab of block rows as scipy
    CSR, the oracle's VankaData of the first chunk[-1] patches (LAPACK
    inverses) with the level's averaging weights, the prolongation; the
    coarsest level's LU factors; a diagonal operator of the finest size."""
    import numpy as np
    import scipy.linalg as sla
    import scipy.sparse as sp
    from oracle import prolongation, to_csr
    from oracle.patches import patch_dofs
    from oracle.vanka import VankaData, local_matrices

    mats = P.system(name)
    cells = [lv.cells for lv in P.levels]
    rng = np.random.default_rng(0)
    levels = []
    for l in range(len(mats) - 1):
        m = mats[l]
        n = m.nrows * m.b
        r1 = min(m.nrows, slab_rows)
        rp = m.rowptr[:r1 + 1].astype(np.int64)
        slab = sp.bsr_matrix((np.asarray(m.vals[:rp[-1]], dtype=np.float64).reshape(-1, m.b, m.b),
                              m.colind[:rp[-1]], rp), shape=(r1 * m.b, n)).tocsr()
        npatch = int(np.prod(cells[l]))
        dofs_all = patch_dofs(cells[l], m.b)
        scale = 1.0 / np.maximum(np.bincount(dofs_all.ravel(), minlength=n), 1.0)
        c = min(chunk[-1], npatch)
        idx = np.arange(c)
        V = VankaData(dofs=dofs_all[idx], inv=np.linalg.inv(local_matrices(m, cells[l], idx)),
                      scale=scale, omega=0.8)
        levels.append(dict(slab=slab, slab_frac=m.nnzb / max(int(rp[-1]), 1), V=V, npatch=npatch,
                           mask=m.dirichlet.astype(bool), x=rng.standard_normal(n),
                           Pm=prolongation(tuple(cells[l + 1]), m.b)))
    mc = mats[-1]
    m0 = mats[0]
    n0 = m0.nrows * m0.b
    return dict(levels=levels, chunk=chunk, lu=sla.lu_factor(to_csr(mc).toarray()),
                rc=rng.standard_normal(mc.nrows * mc.b), D=sp.diags(1.0 + rng.random(n0)).tocsr(),
                b=rng.standard_normal(n0), mask0=m0.dirichlet.astype(bool), n0=n0)


def _oracle_costs(S):
    """Wall time of the FP64 oracle's operations on one system of the
    workload, each timed on the bounded sample of _oracle_setup and scaled to
    the whole level:
      spmv[l]   the oracle's residual product A_l @ x (scipy CSR) on the slab
                of block rows, scaled by nonzero blocks;
      vanka[l]  oracle.vanka_sweep with the residual given (local solves with
                the stored inverses, scatter, update) on two patch counts: the
                slope per patch times the level's patches plus the per-call part;
      R[l], Pr[l]  the oracle's restriction P^T d and prolongation P x (full);
      vec[l]    one whole-vector NumPy pass (x - x) of the level's length;
      coarse    scipy lu_solve of the coarsest level;
      krylov(k) the oracle's FGMRES(20) itself for k iterations on vectors of
                the finest size with a diagonal operator and the identity
                preconditioner (its Gram-Schmidt, rotations, update and true
                residuals), minus those diagonal products."""
    import numpy as np
    import scipy.linalg as sla
    from oracle.fgmres import fgmres
    from oracle.vanka import VankaData, vanka_sweep

    out = {"spmv": [], "vanka": [], "R": [], "Pr": [], "vec": []}
    for lv in S["levels"]:
        x = lv["x"]
        out["spmv"].append(_median_time(lambda: lv["slab"] @ x) * lv["slab_frac"])
        out["vec"].append(_median_time(lambda: x - x))
        V = lv["V"]
        n = x.shape[0]
        z = np.zeros(n)
        ts, cs = [], []
        for c in S["chunk"]:
            c = min(c, V.dofs.shape[0])
            Vc = VankaData(dofs=V.dofs[:c], inv=V.inv[:c], scale=V.scale, omega=V.omega)
            ts.append(_median_time(lambda: vanka_sweep(None, x, z, Vc, lv["mask"], d=x)))
            cs.append(c)
        if cs[-1] > cs[0]:
            slope = max((ts[-1] - ts[0]) / (cs[-1] - cs[0]), 0.0)
            out["vanka"].append(max(ts[0] - slope * cs[0], 0.0) + slope * lv["npatch"])
        else:
            out["vanka"].append(ts[-1] * lv["npatch"] / cs[-1])
        Pm = lv["Pm"]
        xc = x[:Pm.shape[1]]
        out["R"].append(_median_time(lambda: Pm.T @ x))
        out["Pr"].append(_median_time(lambda: Pm @ xc))
    out["coarse"] = _median_time(lambda: sla.lu_solve(S["lu"], S["rc"]))
    out["spmv0"] = out["spmv"][0]
    D, b, n0 = S["D"], S["b"], S["n0"]
    t_diag = _median_time(lambda: D @ b)

    def krylov(k):
        t0 = time.perf_counter()
        fgmres(D, b, np.zeros(n0), lambda v: v.copy(), S["mask0"], rtol=1e-300, maxiter=k, restart=20)
        return max(time.perf_counter() - t0 - (k + 2) * t_diag, 0.0)
    out["krylov"] = krylov
    return out


def _oracle_solve_time(c, iters, nu=(2, 2)):
    """Oracle time of one FGMRES(20) + V-cycle solve with `iters` iterations
    from the per-operation costs c: every iteration runs the V-cycle (per
    smoothing level nu_pre + nu_post Vanka steps, the first with the residual
    given, one residual product per later step and one before the
    restriction, restriction, prolongation, and the cycle's whole-vector
    passes: copy and mask of r, x = 0, the residual subtractions and masks,
    x + P x_c and its mask; the coarse LU solve) and one finest-level product
    A z; the Krylov part is timed as a whole."""
    nu1, nu2 = nu
    vc = c["coarse"]
    for l in range(len(c["spmv"])):
        nres = nu1 - 1 + 1 + nu2
        vc += ((nu1 + nu2) * c["vanka"][l] + nres * c["spmv"][l] + c["R"][l] + c["Pr"][l]
               + (5 + 2 * nres) * c["vec"][l])
    return iters * (vc + c["spmv0"]) + c["krylov"](iters) + 2 * c["spmv0"]


def cpu_baseline(P, iters, n_value):
    """The FP64 oracle timed on the host on a bounded sample of the same
    Newton-step workload (momentum, deformation mass and ALE solves with the
    GPU's iteration counts), once with every host core available to its
    BLAS / LAPACK and once limited to one thread; value = the unknowns of the
    GPU figure / the oracle's step time."""
    import platform
    import threadpoolctl

    systems = [(name, key) for name, key in (("mom", "momentum_iters"), ("mass", "mass_iters"),
                                             ("ale", "ale_iters")) if iters.get(key) is not None]
    t0 = time.perf_counter()
    setup = {name: _oracle_setup(P, name) for name, _ in systems}
    t_setup = time.perf_counter() - t0

    def model():
        t_w, t_c = time.perf_counter(), time.process_time()
        total = 0.0
        parts = {}
        for name, key in systems:
            t = _oracle_solve_time(_oracle_costs(setup[name]), iters[key])
            parts[name] = t
            total += t
        wall = time.perf_counter() - t_w
        cpu = time.process_time() - t_c
        return total, parts, wall, cpu

    model_name = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model_name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    res = {}
    total, parts, wall, cpu = model()
    res["all"] = (total, parts, wall, cpu)
    with threadpoolctl.threadpool_limits(1):
        res["one"] = model()
    t_all, parts_all, wall_all, cpu_all = res["all"]
    t_one, parts_one, wall_one, _ = res["one"]
    return dict(
        value=n_value / t_all, unit="DoF/s", cores=round(cpu_all / wall_all, 1), kind="oracle",
        value_1thread=n_value / t_one,
        step_s=t_all, step_s_1thread=t_one,
        solve_s={k: round(v, 3) for k, v in parts_all.items()},
        host={"cpus": os.cpu_count(), "model": model_name or platform.processor()},
        sample=(f"the oracle's operations on the same workload, each timed on a bounded sample "
                f"and scaled to its level: residual products on slabs of <= 65536 block rows, "
                f"Vanka steps on 2048 and 4096 patches (per-patch slope), full restriction / "
                f"prolongation, the coarse LU solve, and the oracle's FGMRES(20) on finest-size "
                f"vectors; composed with the GPU step's iteration counts "
                f"{ {k: iters.get(k) for k in ('momentum_iters', 'mass_iters', 'ale_iters')} } "
                f"(V-cycle 2/2); {wall_all:.0f} s wall (all cores), {wall_one:.0f} s (1 thread), "
                f"sample set-up {t_setup:.0f} s untimed"))


def run_batched(args):
    """Batched workload: independent 3D instances (N ~ U{16,20,24,32,40},
    random solid box and mu), mixed precision, momentum systems solved to
    1e-8 in lockstep batches that fill an HBM budget (admission waves)."""
    import numpy as np
    import torch
    from fsigen import batch_instance
    from paper_1904_02401_amd import fsimg
    from paper_1904_02401_amd.problems import level_dicts

    prec = fsimg.FSIMG_FP64 if args.only == "fp64" else fsimg.FSIMG_MIXED
    budget = int(args.budget_gb * (1 << 30))
    ctx = fsimg.fsimg_ctx_create(0, budget)
    opts = fsimg.fsimg_default_opts(precision=prec, krylov_lookahead=args.lookahead,
                                    small_level_kib=args.small_level_kib)
    dev = torch.device("cuda:0")
    waves, unknowns, solve_s, sizes, iters = [], 0, 0.0, [], []
    pending = list(range(args.instances))
    check = None
    while pending:
        wave, used, probs = [], 0, []
        while pending:
            P = batch_instance(pending[0])
            fp = fsimg.fsimg_hier_footprint(level_dicts(P, "mom"), opts)
            if wave and used + fp > budget * 0.95:
                break
            pending.pop(0)
            wave.append(P)
            used += fp
        log(f"wave {len(waves)}: {len(wave)} instances, footprint {used / 2**30:.1f} GiB")
        hs = [fsimg.fsimg_hier_create(ctx, level_dicts(P, "mom"), opts) for P in wave]
        for h in hs:
            fsimg.fsimg_factor(h)
        bs = [torch.tensor(P.rhs["mom"], device=dev) for P in wave]
        for rep in range(2):  # warm-up, then timed
            xs = [torch.zeros_like(b) for b in bs]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = fsimg.fsimg_solve_batch(hs, bs, xs)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
        if check is None:  # one instance solved alone must equal its in-batch result
            xa = torch.zeros_like(bs[0])
            fsimg.fsimg_solve(hs[0], bs[0], xa)
            torch.cuda.synchronize()
            check = bool(torch.equal(xa, xs[0]))
        n_w = sum(int(b.numel()) for b in bs)
        unknowns += n_w
        solve_s += t
        waves.append({"instances": len(wave), "unknowns": n_w, "solve_s": t,
                      "footprint_GiB": used / 2**30})
        sizes += [P.levels[0].cells[0] for P in wave]
        iters += [s["iters"] for s in sts]
        for h in hs:
            fsimg.fsimg_hier_destroy(h)
        del hs, bs, xs
    fsimg.fsimg_ctx_destroy(ctx)
    out = {
        "metric": "MG-FGMRES DoF/s + smoother HBM GB/s, FP32-mixed vs FP64 @1e-8; p99 solve latency",
        "value": unknowns / solve_s, "unit": "DoF/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": solve_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if prec == fsimg.FSIMG_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.instances} independent 3D momentum systems, N ~ U{{16,20,24,32,40}}, "
                               "solid box and mu ~ logU[1e4,1e6] per seed, lambda = 4 mu, batched "
                               "FGMRES + V-cycle to 1e-8, admission waves under an HBM budget",
                   "budget_GiB": args.budget_gb, "waves": waves,
                   "iters_min_mean_max": [min(iters), float(np.mean(iters)), max(iters)],
                   "cells_per_axis": sizes, "alone_equals_batched": check,
                   "krylov_lookahead": args.lookahead, "small_level_kib": args.small_level_kib},
    }
    print(json.dumps(out), flush=True)


def serve_once(args, pool, rate, sizes2, sizes3, check_alone):
    """One serving run at one arrival rate on a fresh server; returns the
    figures of that run."""
    import numpy as np
    import torch
    from paper_1904_02401_amd import fsimg

    rng = np.random.Generator(np.random.PCG64(args.seed))
    arrivals, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > args.window:
            break
        d = 2 if rng.uniform() < 0.7 else 3
        sz = int(rng.choice(sizes2 if d == 2 else sizes3))
        ns = rng.integers(3, 6, size=10)
        arrivals.append((t, d, sz, ns))
    ctx = fsimg.fsimg_ctx_create(0, int(args.budget_gb * (1 << 30)))
    opts = fsimg.fsimg_default_opts(precision=fsimg.FSIMG_MIXED)
    nopts = fsimg.fsimg_default_newton_opts(gamma=args.gamma, max_steps=args.max_newton,
                                            lin_rtol=args.lin_rtol, atol=args.newton_atol,
                                            ale_rtol=args.ale_rtol)
    srv = fsimg.fsimg_server_create(ctx, opts, args.max_active)
    fsimg.fsimg_server_set_order(srv, 1 if args.order == "work" else 0)

    def submit(server, key, ns, arrival):
        if args.newton:
            return fsimg.fsimg_server_submit_newton(server, pool[key][0], args.time_steps, nopts, arrival)
        return fsimg.fsimg_server_submit(server, pool[key][0], ns, arrival)
    stream = torch.cuda.current_stream()
    meta, lat, qdelay, done_ids, work, failed, newton_steps = {}, [], [], [], 0.0, [], []
    nxt, steps, max_active_seen = 0, 0, 0
    start = fsimg.fsimg_server_clock(srv)
    last_log = 0.0
    while True:
        now = fsimg.fsimg_server_clock(srv) - start
        while nxt < len(arrivals) and arrivals[nxt][0] <= now:
            ta, d, sz, ns = arrivals[nxt]
            data, nm, na = pool[(d, sz)]
            rid = submit(srv, (d, sz), ns, start + ta)
            meta[rid] = (start + ta, d, sz, nm, na, int(ns.sum()), ns)
            nxt += 1
        active, queued = fsimg.fsimg_server_step(srv, stream)
        steps += 1
        max_active_seen = max(max_active_seen, active)
        for rid, a, f in zip(*fsimg.fsimg_server_poll(srv)):
            arr, d, sz, nm, na, nsteps, _ = meta[abs(int(rid))]
            if rid > 0:
                lat.append(f - arr)
                qdelay.append(a - arr)
                done_ids.append(int(rid))
                if args.newton:  # Newton steps actually taken over the request's time steps
                    nsteps = fsimg.fsimg_server_newton_stats(srv, int(rid))["steps"]
                    newton_steps.append(nsteps)
                work += nsteps * (nm + na)
            else:
                st = fsimg.fsimg_server_request_status(srv, abs(int(rid)))
                failed.append({"dim": d, "cells": sz, "status": st})
                log(f"  request {abs(int(rid))} ({d}D {sz}^{d}) failed with status {st}")
        now = fsimg.fsimg_server_clock(srv) - start
        if now - last_log > 10.0:
            last_log = now
            log(f"  rate {rate}/s t={now:.1f} s: {nxt} arrived, {active} running, {queued} queued, "
                f"{len(lat)} completed")
        if nxt >= len(arrivals) and active == 0 and queued == 0:
            break
        if now > args.max_wall:
            log(f"  rate {rate}/s: stopped at {now:.1f} s with {active} running, {queued} queued")
            break
        if active == 0 and nxt < len(arrivals):
            time.sleep(max(0.0, min(arrivals[nxt][0] - now, 0.05)))
    wall = fsimg.fsimg_server_clock(srv) - start
    same = None
    if check_alone and done_ids:
        # a completed request served again alone must give the same result
        rid = done_ids[len(done_ids) // 2]
        arr, d, sz, nm, na, nsteps, ns = meta[rid]
        xm_mix, xa_mix = fsimg.fsimg_server_result(srv, rid, nm, na)
        srv2 = fsimg.fsimg_server_create(ctx, opts)
        rid2 = submit(srv2, (d, sz), ns, fsimg.fsimg_server_clock(srv2))
        while True:
            act, q = fsimg.fsimg_server_step(srv2, stream)
            if act == 0 and q == 0:
                break
        fsimg.fsimg_server_poll(srv2)
        xm_al, xa_al = fsimg.fsimg_server_result(srv2, rid2, nm, na)
        same = bool(np.array_equal(xm_mix, xm_al) and np.array_equal(xa_mix, xa_al))
        fsimg.fsimg_server_destroy(srv2)
    fsimg.fsimg_server_destroy(srv)
    fsimg.fsimg_ctx_destroy(ctx)
    lat_a = np.array(lat) if lat else np.array([np.nan])
    q_a = np.array(qdelay) if qdelay else np.array([np.nan])
    return {"rate_req_s": rate, "arrived": len(arrivals), "completed": len(lat),
            "offered_req_s": len(arrivals) / args.window, "achieved_req_s": len(lat) / wall,
            "wall_s": wall, "server_steps": steps, "max_running": max_active_seen,
            "dof_per_s": work / wall,
            "latency_p50_s": float(np.percentile(lat_a, 50)),
            "latency_p99_s": float(np.percentile(lat_a, 99)),
            "queue_delay_p50_s": float(np.percentile(q_a, 50)),
            "queue_delay_p99_s": float(np.percentile(q_a, 99)),
            "alone_equals_mix": same, "failed": failed,
            "newton_steps_per_request": (float(np.mean(newton_steps)) if newton_steps else None)}


def run_serving(args):
    """Serving workload: Poisson arrivals of FSI simulations (10 time steps of
    3..5 Newton steps, or with --newton --time-steps real Newton time steps
    on the GPU; 70 % 2D 64^2..256^2, 30 % 3D 16^3..48^3), hierarchies
    resident in HBM, first-fit admission by footprint, continuous batching,
    mixed precision.  Latency = arrival -> last solve of the simulation.
    --rates runs a sweep of arrival rates on the same request pool."""
    from fsigen import serve_request
    from paper_1904_02401_amd.problems import request_data

    sizes2 = (64, 80, 96, 128, 160, 192, 256)
    sizes3 = tuple(n for n in (16, 20, 24, 32, 40, 48) if n <= args.max3d)
    t0 = time.perf_counter()
    import torch
    pinned = []

    def pin(a):
        # momentum values are uploaded again at every change of state: keep
        # them in page-locked host memory so that the copies run at DMA speed
        t = torch.empty(a.shape, dtype=torch.float64, pin_memory=True)
        t.numpy()[...] = a
        pinned.append(t)
        return t.numpy()

    pool = {}
    for d, sz in [(2, n) for n in sizes2] + [(3, n) for n in sizes3]:
        if args.newton:
            from fsigen import serve_instance
            from paper_1904_02401_amd import fsimg
            from paper_1904_02401_amd.problems import fsi_levels, fsi_state, level_dicts
            P = serve_instance(d, sz, seed=sz)
            pool[(d, sz)] = (fsimg.NewtonRequestData(level_dicts(P, "mom"), level_dicts(P, "ale"),
                                                     fsi_levels(P), P.params, *fsi_state(P)),
                             P.levels[0].systems["mom"].nrows * (d + 1),
                             P.levels[0].systems["ale"].nrows * d)
            log(f"  pool: {d}D {sz}^{d}, {len(P.levels)} levels, Newton request")
            continue
        P, states, rhs = serve_request(d, sz, seed=sz, n_states=args.n_states, n_rhs=args.n_rhs)
        if args.n_states > 1:
            for prob in [P] + states:
                for lv in prob.levels:
                    lv.systems["mom"].vals = pin(lv.systems["mom"].vals)
        log(f"  pool: {d}D {sz}^{d}, {len(P.levels)} levels, {1 + len(states)} states, "
            f"{1 + len(rhs)} right-hand sides")
        pool[(d, sz)] = (request_data(P, states, rhs), P.levels[0].systems["mom"].nrows * (d + 1),
                         P.levels[0].systems["ale"].nrows * d)
    log(f"serving pool of {len(pool)} simulations generated in {time.perf_counter() - t0:.1f} s")
    rates = [float(r) for r in args.rates.split(",")] if args.rates else [args.rate]
    runs = []
    for k, rate in enumerate(rates):
        runs.append(serve_once(args, pool, rate, sizes2, sizes3, check_alone=(k == len(rates) - 1)))
        log(f"rate {rate}/s: {json.dumps(runs[-1])}")
    main = runs[-1]
    out = {
        "metric": "MG-FGMRES DoF/s + smoother HBM GB/s, FP32-mixed vs FP64 @1e-8; p99 solve latency",
        "value": main["dof_per_s"], "unit": "DoF/s", "n_gpus": 1, "steps": main["server_steps"],
        "warmup": 0, "ms_per_step": main["wall_s"] / max(main["server_steps"], 1) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": (
            ("serving: Poisson arrivals of FSI simulations, " + (
                f"{args.time_steps} Newton time steps each on the GPU (residual and Jacobian "
                f"assembly, reuse with gamma_nt = {args.gamma}, line search; Newton stop at 1e-8 "
                f"relative or {args.newton_atol:g} absolute, at most {args.max_newton} Newton steps per "
                f"time step, momentum solves to {args.lin_rtol:g}, ALE solves to 1e-8, batched across "
                "requests), "
                if args.newton else
                "10 time steps x 3..5 Newton steps (momentum + deformation + ALE solves to 1e-8; a new "
                "Jacobian state uploaded and refactored every time step, a new right-hand side every "
                "Newton step), ") +
            f"70% 2D 64^2..256^2, 30% 3D 16^3..{max(sizes3)}^3, mixed precision, resident "
            "hierarchies, first-fit admission by HBM footprint, continuous batching")),
                   "window_s": args.window, "budget_GiB": args.budget_gb,
                   "max_active": args.max_active, "admission_order": args.order,
                   "states_cycled": args.n_states,
                   "rhs_cycled": args.n_rhs, **main},
    }
    if len(runs) > 1:
        out["sweep"] = runs
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--mu", type=float, default=None, help="solid shear modulus override")
    ap.add_argument("--lam", type=float, default=None, help="solid Lame lambda override")
    ap.add_argument("--omega", type=float, default=0.8,
                    help="Vanka damping omega_V (the paper's 0.8)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-tune", action="store_true", help="built-in launch shapes, no tuning")
    ap.add_argument("--schedule", choices=["gather", "parity", "greedy", "auto"], default="gather",
                    help="Vanka schedule: per-dof gather (batched path), coloured scatter, or "
                         "auto (time all three per system at setup, use the fastest)")
    ap.add_argument("--patches", choices=["element", "block"], default=None,
                    help="Vanka patches: one element, or 2x2(x2) element blocks (3D: solid only); "
                         "default element, block on the benchmark channel")
    ap.add_argument("--smoother", choices=["vanka", "ilu"], default="vanka",
                    help="multigrid smoother (ilu: block ILU(0), level-scheduled)")
    ap.add_argument("--no-mass", action="store_true")
    ap.add_argument("--lookahead", type=int, choices=[1, 2], default=2,
                    help="FGMRES iterations the host keeps in flight (1: wait for each)")
    ap.add_argument("--small-level-kib", type=int, default=0,
                    help="levels up to this many KiB of smoother + matrix data run in one "
                         "workgroup per instance (0: a launch per step and level)")
    ap.add_argument("--newton", action="store_true",
                    help="time steps of the GPU Newton loop (residual / Jacobian assembly, reuse, "
                         "line search) instead of one linear Newton-step solve")
    ap.add_argument("--gamma", type=float, default=0.05, help="Newton: Jacobian reuse threshold")
    ap.add_argument("--lin-rtol", type=float, default=1e-4,
                    help="Newton: relative tolerance of each momentum solve (the paper: 1e-4)")
    ap.add_argument("--ale-rtol", type=float, default=None,
                    help="Newton: tolerance of the ALE solves (0: the ALE hierarchy's 1e-8; "
                         "default 1e-4 on the benchmark channel, 0 elsewhere)")
    ap.add_argument("--newton-atol", type=float, default=1e-8,
                    help="Newton: absolute max-norm stop (the paper: 1e-8, besides the relative 1e-8)")
    ap.add_argument("--time-steps", type=int, default=1,
                    help="serving with --newton: Newton time steps per request")
    ap.add_argument("--max-newton", type=int, default=50,
                    help="serving with --newton: Newton steps per time step at most")
    ap.add_argument("--chain", action="store_true",
                    help="Newton: successive time steps (warm-up ones included), each from the last "
                         "converged state with the Jacobian carried over")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None,
                    help="run one precision only (profiling runs)")
    ap.add_argument("--kernels-only", type=int, default=0, metavar="REPS",
                    help="only launch REPS finest-level smoothing steps (counter runs)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device copies of MIB MiB (counter calibration)")
    ap.add_argument("--instances", type=int, default=64, help="batched workload size")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="HBM budget of the batched workload")
    ap.add_argument("--rate", type=float, default=20.0, help="serving: mean arrivals per second")
    ap.add_argument("--rates", default="", help="serving: comma-separated arrival-rate sweep")
    ap.add_argument("--window", type=float, default=3.0, help="serving: arrival window (s)")
    ap.add_argument("--max-wall", type=float, default=200.0,
                    help="serving: stop after this many s (long enough for rate 20 to complete every request)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--max-active", type=int, default=0,
                    help="serving: admitted requests at most (0 = as many as fit)")
    ap.add_argument("--n-states", type=int, default=2,
                    help="serving: Jacobian states cycled over a request's time steps")
    ap.add_argument("--n-rhs", type=int, default=3,
                    help="serving: momentum right-hand sides cycled over a request's Newton steps")
    ap.add_argument("--max3d", type=int, default=48, help="serving: largest 3D mesh (cells per axis)")
    ap.add_argument("--order", choices=["arrival", "work"], default="arrival",
                    help="serving: admission in arrival order or least work first")
    args = ap.parse_args()
    if args.ale_rtol is None:
        args.ale_rtol = 1e-4 if args.config in CHANNEL_CONFIGS else 0.0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              f"sharding of this path is not built", file=sys.stderr)
        sys.exit(2)
    if args.config == "c4":
        run_batched(args)
        return
    if args.config == "c5":
        run_serving(args)
        return
    if args.calib_copy:
        calib_copy(args.calib_copy << 20, 5)
        return
    if args.config in CHANNEL_CONFIGS:
        run_channel(args)
        return
    args.patches = args.patches or "element"
    import numpy as np
    from fsigen import config_problem
    from oracle import to_csr

    t0 = time.perf_counter()
    over = {}
    if args.mu is not None:
        over["mu_s"] = args.mu
    if args.lam is not None:
        over["lambda_s"] = args.lam
    P = config_problem(args.config, seed=0, params=over or None)
    log(f"problem {args.config} generated in {time.perf_counter() - t0:.1f} s")
    from paper_1904_02401_amd import fsimg
    if args.kernels_only:
        kernels_only(P, fsimg.FSIMG_MIXED if args.only == "mixed" else fsimg.FSIMG_FP64,
                     args.kernels_only)
        return
    if args.newton:
        run_newton(args, P)
        return
    lev = P.levels[0]
    n_mom = lev.systems["mom"].nrows * lev.systems["mom"].b
    n_ale = lev.systems["ale"].nrows * lev.systems["ale"].b
    runs = {}
    precs = [("mixed", fsimg.FSIMG_MIXED), ("fp64", fsimg.FSIMG_FP64)]
    if args.only:
        precs = [p for p in precs if p[0] == args.only]
    elif args.no_fp64:
        precs = precs[:1]
    for tag, prec in precs:
        r = run_gpu(P, prec, args.steps, args.warmup, with_mass=not args.no_mass, tune=not args.no_tune,
                    patches=fsimg.FSIMG_PATCH_BLOCK if args.patches == "block" else fsimg.FSIMG_PATCH_ELEMENT,
                    schedule={"gather": fsimg.FSIMG_VANKA_GATHER, "parity": fsimg.FSIMG_VANKA_PARITY,
                              "greedy": fsimg.FSIMG_VANKA_GREEDY, "auto": -1}[args.schedule],
                    smoother=fsimg.FSIMG_SMOOTHER_ILU if args.smoother == "ilu" else fsimg.FSIMG_SMOOTHER_VANKA,
                    lookahead=args.lookahead, small_kib=args.small_level_kib, omega=args.omega)
        A = to_csr(lev.systems["mom"])
        mask = lev.systems["mom"].dirichlet.astype(bool)
        rr = P.rhs["mom"] - A @ r["x_mom"]
        rr[mask] = 0.0
        r["rel_res_host"] = float(np.linalg.norm(rr) / np.linalg.norm(P.rhs["mom"]))
        Aa = to_csr(lev.systems["ale"])
        amask = lev.systems["ale"].dirichlet.astype(bool)
        ra = P.rhs["ale"] - Aa @ r["x_ale"]
        ra[amask] = 0.0
        r["rel_res_ale_host"] = float(np.linalg.norm(ra))  # relative to ||r0|| below
        runs[tag] = r
        st_m, st_s, st_a = r["stats"]
        if st_m["status"] != fsimg.FSIMG_OK:
            log(f"{tag}: the momentum solve did not converge ({st_m['iters']} iterations, "
                f"rel. residual {st_m['rel_res']:.2e}); the figures below are not a valid step")
        log(f"{tag}: {r['t_step'] * 1e3:.2f} ms/step, momentum {st_m['iters']} it "
            f"(rel res {r['rel_res_host']:.2e} host), ALE {st_a['iters']} it, "
            f"mass {st_s['iters'] if st_s else '-'} it; setup {r['t_setup']:.2f} s, "
            f"factor {r['t_factor']:.2f} s")
    def kernel_rates(R, tag):
        s = 8 if tag == "fp64" else 4
        info = R["info_m"]
        prof = R["prof"]
        v_ms = sum(p["vanka_ms"] for p in prof)
        v_n = sum(p["vanka_launches"] for p in prof)
        s_ms = sum(p["spmv_ms"] for p in prof)
        s_n = sum(p["spmv_launches"] for p in prof)
        nl = 27 if P.dim == 3 else 9
        vb = vanka_bytes(info["npatch"], info["np"], nl, s)
        sb = spmv_bytes(info["nnzb"], info["nrows"], lev.systems["mom"].b, s)
        v_avg = v_ms / max(v_n, 1) * 1e-3
        s_avg = s_ms / max(s_n, 1) * 1e-3
        tname = "double" if tag == "fp64" else "float"
        bm = lev.systems["mom"].b
        rpw = R["shapes"].get("mom/L0", {}).get("spmv_rows_per_wave", 1)
        out = {"vanka_patch": {"kernel": f"kb_vanka_patch<{tname}>",
                               "GB/s": vb / v_avg / 1e9 if v_n else 0.0, "avg_ms": v_avg * 1e3,
                               "launches": v_n, "bytes_per_launch": vb, "total_ms": v_ms},
               "spmv_residual": {"kernel": f"kb_spmv<{bm}, {tname}, 0, {rpw}>",
                                 "GB/s": sb / s_avg / 1e9 if s_n else 0.0, "avg_ms": s_avg * 1e3,
                                 "launches": s_n, "bytes_per_launch": sb, "total_ms": s_ms}}
        # transfers between the finest and the next level: (N_f + N_c) b s read / written
        # by the restriction, (2 N_f + N_c) b s by the prolongation, plus the masks
        nf = lev.systems["mom"].nrows * bm
        nc = P.levels[1].systems["mom"].nrows * bm
        rname = f"kb_restrict3<{bm}, {tname}>" if P.dim == 3 else f"kb_restrict<{bm}, 2, {tname}>"
        for key, kname, byts in (("restrict", rname, (nf + nc) * s + nc),
                                 ("prolong", f"kb_prolong<{bm}, {P.dim}, {tname}>", (2 * nf + nc) * s + nf)):
            ms = sum(p[f"{key}_ms"] for p in prof)
            n = sum(p[f"{key}_launches"] for p in prof)
            avg = ms / max(n, 1) * 1e-3
            out[key] = {"kernel": kname, "GB/s": byts / avg / 1e9 if n else 0.0, "avg_ms": avg * 1e3,
                        "launches": n, "bytes_per_launch": byts, "total_ms": ms}
        return out

    def factor_rate(R, tag):
        # algorithmic flops of inverting one n_p x n_p matrix: 2 n_p^3
        info = R["info_m"]
        if args.patches != "element" or args.smoother != "vanka" or not R["factor_ms"]:
            return None
        ms = sum(R["factor_ms"]) / len(R["factor_ms"])
        flops = info["npatch"] * 2.0 * info["np"] ** 3
        nt = (info["np"] + 15) // 16
        tf = flops / (ms * 1e-3) / 1e12
        return {"kernel": f"k_patch_factor_mfma<{nt}, {'double' if tag == 'fp64' else 'float'}>",
                "bound": "mfma", "achieved": tf, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / FP64_MFMA_PEAK_TFLOPS, "flops_per_launch": flops, "avg_launch_ms": ms,
                "launches": len(R["factor_ms"]), "patches": info["npatch"], "n_p": info["np"]}

    def latency(R):
        """p50 / p99 over the timed steps: the whole Newton-step solve
        (momentum, deformation update, mass and ALE solves) and each solve"""
        def pct(v):
            v = np.asarray(v, dtype=np.float64)
            return {"p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99)),
                    "max": float(v.max()), "n": int(v.size)} if v.size else None
        out = {"step": pct([t * 1e3 for t in R["lat"]])}
        for k, v in R["solve_ms"].items():
            out[f"{k}_solve"] = pct(v)
        return out

    def solve_bandwidth(R):
        """each solve's algorithmic device-memory bytes (fsimg_stats.bytes_moved:
        every matrix, inverse, index and vector entry its kernels must touch)
        over its wall time, against the 8 TB/s peak"""
        out = {}
        for j, k in enumerate(("mom", "mass", "ale")):
            st = R["stats"][j]
            if st is None or st["solve_ms"] <= 0:
                continue
            gbs = st["bytes_moved"] / (st["solve_ms"] * 1e-3) / 1e9
            out[k] = {"bytes": st["bytes_moved"], "ms": st["solve_ms"], "GB/s": gbs,
                      "frac": gbs / HBM_PEAK_GBS}
        return out

    main_tag = precs[0][0]
    R = runs[main_tag]
    kr = kernel_rates(R, main_tag)
    role = max(("vanka_patch", "spmv_residual"), key=lambda k: kr[k]["total_ms"])
    dom = kr[role]
    traffic = measured_traffic(role, f"{args.config}-momentum-level0", main_tag)
    value = (n_mom + n_ale) / R["t_step"]
    out = {
        "metric": "MG-FGMRES DoF/s + smoother HBM GB/s, FP32-mixed vs FP64 @1e-8; p99 solve latency",
        "value": value,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["t_step"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_tag == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": {
            "c1": ("2D [0,1]^2, solid [0.3,0.7]x[0.45,0.55], 32^2 Q2 quads, 3 MG levels, "
                   "momentum (p,v) + deformation + ALE solves to rel. residual 1e-8"),
            "c2": ("3D [0,1]^3, solid [0.3,0.7]x[0.4,0.6]^2, 32^3 Q2 hexes, 4 MG levels, "
                   "momentum (p,v) + deformation + ALE solves to rel. residual 1e-8"),
            "c3": ("3D [0,1]^3, solid [0.3,0.7]x[0.4,0.6]^2, 64^3 Q2 hexes, 5 MG levels, "
                   "momentum (p,v) + deformation + ALE solves to rel. residual 1e-8")}.get(
                       args.config, args.config),
                   "mu_s": P.params["mu_s"], "lambda_s": P.params["lambda_s"],
                   "unknowns_momentum": n_mom, "unknowns_ale": n_ale,
                   "precision": main_tag, "vanka_patches": args.patches,
                   "vanka_schedule": args.schedule, "smoother": args.smoother, "omega_vanka": args.omega,
                   "krylov_lookahead": args.lookahead, "small_level_kib": args.small_level_kib},
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["GB/s"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["GB/s"] / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": dom["bytes_per_launch"],
                     "avg_launch_ms": dom["avg_ms"], "launches": dom["launches"]},
        "kernels": {k: dict(v, traffic=measured_traffic(k, f"{args.config}-momentum-level0", main_tag))
                    for k, v in kr.items()},
        "patch_factor": factor_rate(R, main_tag),
        "latency_ms": latency(R),
        "solve_bandwidth": solve_bandwidth(R),
        "solve": {"momentum_converged": R["stats"][0]["status"] == fsimg.FSIMG_OK,
                  "momentum_status": R["stats"][0]["status"],
                  "momentum_rel_res_device": R["stats"][0]["rel_res"],
                  "momentum_res_hist": R["stats"][0]["res_hist"],
                  "momentum_iters": R["stats"][0]["iters"], "ale_iters": R["stats"][2]["iters"],
                  "mass_iters": R["stats"][1]["iters"] if R["stats"][1] else None,
                  "rel_res_momentum_fp64_host": R["rel_res_host"],
                  "setup_s": R["t_setup"], "factor_s": R["t_factor"], "tune_s": R["t_tune"],
                  "launch_shapes": R["shapes"],
                  "schedule_ms_per_vcycle": R["schedule_ms"] or None},
    }
    if "fp64" in runs and main_tag != "fp64":
        F = runs["fp64"]
        out["fp64"] = {"value": (n_mom + n_ale) / F["t_step"], "ms_per_step": F["t_step"] * 1e3,
                       "latency_ms": latency(F), "solve_bandwidth": solve_bandwidth(F),
                       "momentum_iters": F["stats"][0]["iters"], "ale_iters": F["stats"][2]["iters"],
                       "rel_res_momentum_fp64_host": F["rel_res_host"],
                       "kernels": kernel_rates(F, "fp64")}
        out["mixed_speedup_vs_fp64"] = F["t_step"] / R["t_step"]
        out["mixed_rel_err_vs_fp64"] = _split_err(R["x_mom"], F["x_mom"], P.dim + 1)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(P, out["solve"], n_mom + n_ale)
    log(f"peak host RSS {resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 1e6:.1f} GB")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
