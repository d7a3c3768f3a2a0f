#!/usr/bin/env python3
"""Benchmark: FMM-BEM matvecs/s on the 81920-element unit sphere at k = 8.

One timed step is one full solve of the Burton-Miller system for a plane
wave (direction drawn from the workload seed) to a true float64 relative
residual of 1e-6, with the float32 FMM operator inside GMRES and float64
residuals / corrections outside (iterative refinement).  ``value`` is the
effective throughput: the number of float64 FMM matvecs that plain float64
GMRES(50) needs for the same solve, divided by the mixed-precision solve's
wall time.  Plan construction (tree, near field, operators) happens before
the timed region; all inputs are resident in device memory.

Also reported: plain float64 and float32 matvecs/s, per-stage times from HIP
events on the library's stream, the roofline of the dominant kernel, and the
CPU oracle timed on a bounded sample of rows.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

``--workload batch32`` times the mixed-mesh batch instead: 16 state and 16
adjoint solves over icosphere levels 4/5/6 and k in {2, 4, 8} (nine
problems, leaf levels tuned at plan creation) through one lockstep batched
solve; its line reports solves/s and the same 32 solves run one by one.

``--workload grad_cube49152_k6`` times the objective and its gradient on
the 49152-element cube surface at k = 6: J = sum |p(x_m)|^2 over 8 points on
the radius-3 sphere and dJ/dbeta for a per-element admittance beta, i.e. a
state solve, the field at the points, an adjoint solve and the gradient,
both solves in mixed precision to a float64 residual of 1e-6.

``--workload elastic_sphere`` times the BEM-FEM coupled solve of the paper's
elastic-sphere benchmark (tungsten sphere of radius 0.25 in water, omega =
1, 3211 finite-element nodes, 1280 boundary triangles): BEM plan, FEM
assembly, LU and coupling matrix, GMRES to 1e-5; its line reports solves/s
and the parts.

``--workload topo_sphere81920_k8`` times the topological derivative T_Omega
on the design-domain lattice (101^3 points on [-1.25, 1.25]^3, those outside
the sphere): state and adjoint fields and gradients at the points by the
FMM, then T_Omega; its line reports lattice points/s.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12   # MI355X dense matrix FP32 (FLOP/s)
PEAK_FP64 = 78.6e12         # MI355X FP64 vector / matrix
PEAK_FP32_VEC = 157.3e12
HBM_PEAK = 8.0e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(V, T, k, seed, target_s=15.0):
    """Oracle matrix-free matvec on sampled rows, process-parallel; returns
    (matvecs/s, cores, rows)."""
    import multiprocessing as mp

    from oracle import bem as obem
    # every core this process may run on, up to 16 (the host-CPU share of one
    # GPU on the benchmark machines: more worker processes there would only
    # queue behind each other)
    cores = min(len(os.sched_getaffinity(0)), 16)
    geom = obem.Geometry(V, T)
    n = geom.n_elem
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    rows_all = rng.permutation(n)
    # calibrate with one small block (single process)
    t0 = time.perf_counter()
    obem.matvec(geom, k, 1j / k, p, None, rows=rows_all[:16], block=16)
    per_row = (time.perf_counter() - t0) / 16
    nrows = int(max(cores * 8, min(n, target_s * cores / max(per_row, 1e-6))))
    nrows = min(nrows, n)
    chunks = np.array_split(rows_all[:nrows], cores * 4)
    ctx = mp.get_context("fork")
    global _G
    _G = (geom, k, p)
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_cpu_rows, chunks)
    dt = time.perf_counter() - t0
    return nrows / (n * dt), cores, nrows, dt


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_G = None


def measured_traffic():
    """HBM bytes per float32 M2L launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "m2l_counters.json")
    try:
        meta = json.load(open(path))
        src = open(os.path.join(ROOT, meta["kernel_source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != meta.get("kernel_source_sha256"):
        return None
    return meta.get("bytes_per_launch")


def _cpu_rows(rows):
    import os as _os
    _os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import bem as obem
    geom, k, p = _G
    obem.NEAR_WORKERS = 1   # near integrals inside this worker, no nested pool
    return obem.matvec(geom, k, 1j / k, p, None, rows=rows, block=16)


def run_batch(args):
    """Mixed-mesh batch of 32 solves (16 state, 16 adjoint), mixed precision."""
    import torch

    import paper_1606_02383_amd as bem
    from workloads import batch32, icosphere

    cases, obs = batch32()
    combos = sorted({(lvl, k) for lvl, k, _ in cases})
    meshes = {lvl: icosphere(lvl) for lvl in sorted({c[0] for c in combos})}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = bem.Plan([bem.Problem(*meshes[lvl], k, leaf_cap=64, leaf_level=-1)
                     for lvl, k in combos])
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    index = {c: i for i, c in enumerate(combos)}
    for i, (lvl, k) in enumerate(combos):
        st = plan.stats(i)
        log(f"[bench] problem {i}: level {lvl} n={st['n_tri']} k={k} leaf level "
            f"{st['leaf_level']} ({st['tuned_ms']:.3f} ms per float32 product), schedule "
            f"{st['schedule']}, direct depth {st['direct_depth']}")
    log(f"[bench] plan of {len(combos)} problems built (with tuning) in {t_plan:.2f} s")
    opts = bem.GmresOptions(tol=1e-6, restart=50, mode=1, inner_tol=args.inner_tol)
    systems = []
    for lvl, k, d in cases:
        pr = index[(lvl, k)]
        systems.append(dict(prob=pr, b=plan.plane_wave_rhs(d, prob=pr)))
    # adjoint right-hand sides of J = sum |p(x_obs)|^2 from the state solutions
    # (set-up, outside the timed region)
    xs, _ = plan.solve_batch(systems, opts)
    for s_, (lvl, k, d) in enumerate(cases):
        pr = index[(lvl, k)]
        pobs = plan.eval_field(xs[s_], None, obs, direction=d, prob=pr)
        rp, _ = plan.eval_field_adjoint(obs, pobs, prob=pr)
        systems.append(dict(prob=pr, b=rp, adjoint=True))
    for _ in range(args.warmup):
        plan.solve_batch(systems, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xs, infos = plan.solve_batch(systems, opts)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    assert all(i["converged"] and i["resid"] <= 1e-6 for i in infos), infos
    mv32 = sum(i["matvec32"] for i in infos)
    mv64 = sum(i["matvec64"] for i in infos)
    log(f"[bench] batch: {dt * 1e3:.1f} ms per 32 solves, {mv32} float32 + {mv64} float64 "
        f"products, worst resid {max(i['resid'] for i in infos):.2e}")
    # the same 32 solves one after another on the caller's stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sy in systems:
        plan.solve(sy["b"], adjoint=sy.get("adjoint", False), opts=opts, prob=sy["prob"])
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    log(f"[bench] one by one: {dt_seq * 1e3:.1f} ms")
    out = {
        "metric": "batched BEM solves/sec (16 state + 16 adjoint, mixed meshes, FP32+refine, "
                  "rel resid 1e-6)",
        "value": len(systems) / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64+c128", "data": "synthetic",
        "config": {"workload": "batch32", "problems": [f"ico{l} k={k}" for l, k in combos],
                   "systems": "16 state (plane waves) + 16 adjoint (J over 8 points, r=3)",
                   "tol": 1e-6, "inner_tol": args.inner_tol, "leaf_level": "tuned"},
        "matvecs_per_step": {"f32": mv32, "f64": mv64},
        "matvecs_per_s": (mv32 + mv64) / dt,
        "sequential_ms": dt_seq * 1e3, "batch_speedup": dt_seq / dt,
        "plan_build_s": t_plan,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_grad(args):
    """Objective and admittance gradient on the cube (state + adjoint solve)."""
    import torch

    import paper_1606_02383_amd as bem
    from workloads import WORKLOADS, admittance, unit_directions

    wl = WORKLOADS["cube49152_k6"]
    V, T = wl.mesh_arrays()
    rng = np.random.default_rng(wl.seed)
    beta = torch.from_numpy(admittance(rng, len(T))).cuda()
    d = unit_directions(rng, 1)[0]
    pts = 3.0 * unit_directions(rng, 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = bem.Plan(bem.Problem(V, T, wl.k, leaf_cap=64))
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    opts = bem.GmresOptions(tol=1e-6, restart=50, mode=1, inner_tol=args.inner_tol)
    for _ in range(args.warmup):
        plan.objective_grad(beta, d, pts, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        J, grad, _, fi, ai = plan.objective_grad(beta, d, pts, opts)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    mv32 = fi["matvec32"] + ai["matvec32"]
    mv64 = fi["matvec64"] + ai["matvec64"]
    log(f"[bench] gradient: {dt * 1e3:.1f} ms per J + dJ/dbeta (J = {J:.6e}); state "
        f"{fi['matvec32']} + {fi['matvec64']}, adjoint {ai['matvec32']} + {ai['matvec64']} "
        f"float32 + float64 products; residuals {fi['resid']:.2e}, {ai['resid']:.2e}")
    out = {
        "metric": "objective + gradient evaluations/sec (J and dJ/dbeta: state and adjoint "
                  "solve, cube N=49152, k=6, FP32+refine, rel resid 1e-6)",
        "value": 1.0 / dt, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64+c128", "data": "synthetic",
        "config": {"workload": "grad_cube49152_k6", "n_tri": len(T), "k": wl.k,
                   "objective": "sum |p|^2 over 8 points on the radius-3 sphere",
                   "admittance": "per element, Re and Im uniform on [0, 0.5]",
                   "tol": 1e-6, "inner_tol": args.inner_tol},
        "matvecs_per_step": {"f32": mv32, "f64": mv64},
        "plan_build_s": t_plan,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_elastic(E, nodes, tets, V, T, alpha):
    """The oracle's whole elastic-sphere solve (dense BEM blocks, dense
    coupling matrix of the body, LU of the coupled system); returns
    (solves/s, threads, seconds)."""
    from oracle import bem as obem
    from oracle import fem
    threads = min(len(os.sched_getaffinity(0)),
                  int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0)))))
    t0 = time.perf_counter()
    g = obem.Geometry(V, T)
    Mp, Mq = obem.bm_blocks(g, E.omega, alpha)
    C = fem.coupling_matrix(nodes, tets, T, E.lam, E.mu, E.rho_s, E.rho_f, E.omega)
    b = obem.plane_wave_rhs(g, E.omega, alpha, np.array(E.direction))
    np.linalg.solve(fem.coupled_operator(Mp, Mq, C), b)
    dt = time.perf_counter() - t0
    return 1.0 / dt, threads, dt


def run_elastic(args):
    """The elastic-sphere benchmark of the BEM-FEM coupling (Sec. 3.1): one
    step is the whole solve the paper times for it -- the BEM plan of the
    sphere's surface, the FEM assembly and factorisation of the body with
    the coupling matrix C, and GMRES on the coupled operator to a relative
    residual of 1e-5 (float64)."""
    import torch

    import paper_1606_02383_amd as bem
    from workloads import ELASTIC_SPHERE as E

    nodes, tets, V, T = E.mesh()
    n = len(T)
    d = np.array(E.direction)
    # the paper's numerical examples: FMM truncation and GMRES tolerance 1e-5;
    # its coupled operator (Eq. GMRES) is the conventional one, alpha = 0 (the
    # sphere at k R = 0.25 lies far below the first fictitious frequency,
    # k R = pi)
    fmm_tol = 1e-5
    alpha = 0.0
    opts = bem.GmresOptions(tol=1e-5, restart=50, mode=0)
    log(f"[bench] elastic sphere: {len(nodes)} nodes ({3 * len(nodes)} unknowns), "
        f"{len(tets)} tetrahedra, {n} boundary triangles, omega = {E.omega}")

    def step():
        t0 = time.perf_counter()
        plan = bem.Plan(bem.Problem(V, T, E.omega, alpha=alpha, fmm_tol=fmm_tol))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cp = bem.Coupling(plan, nodes, tets, T, E.lam, E.mu, E.rho_s, E.rho_f, E.omega)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        x, info = cp.solve(plan.plane_wave_rhs(d), opts=opts)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return (t1 - t0, t2 - t1, t3 - t2), plan, cp, info

    for _ in range(args.warmup):
        _, plan, cp, _ = step()
        cp.close()
        plan.close()
    parts = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts, plan, cp, info = step()
        parts.append(ts)
        if i + 1 < args.steps:
            cp.close()
            plan.close()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    plan_s, coup_s, solve_s = (float(np.mean([p[i] for p in parts])) for i in range(3))
    ndof = 3.0 * len(nodes)
    lu_flop = 2.0 / 3.0 * ndof ** 3 + 2.0 * ndof ** 2 * n
    log(f"[bench] elastic sphere: {dt * 1e3:.1f} ms per solve: plan {plan_s * 1e3:.1f}, "
        f"coupling (assembly, LU, C) {coup_s * 1e3:.1f}, GMRES {solve_s * 1e3:.2f} ms "
        f"({info['iterations']} iterations, residual {info['resid']:.2e})")
    # the adjoint problem on the same plan and coupling (no new factorisation,
    # Sec. 2.5): GMRES on the conjugate-transposed coupled operator
    b_adj = plan.plane_wave_rhs(d)
    cp.solve(b_adj, adjoint=True, opts=opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, ainfo = cp.solve(b_adj, adjoint=True, opts=opts)
    torch.cuda.synchronize()
    adj_s = time.perf_counter() - t0
    log(f"[bench] adjoint solve on the same coupling: {adj_s * 1e3:.2f} ms "
        f"({ainfo['iterations']} iterations)")
    # the dense coupling product alone (one kernel per call, 8 n^2 bytes of C
    # per launch): 200 launches captured in a HIP graph and replayed between
    # two HIP events on the stream, so that the launches run back to back
    # (calls from Python one by one would time the host's launch rate)
    p = torch.ones(n, dtype=torch.complex128, device="cuda")
    for _ in range(10):
        cp.apply(p)
    torch.cuda.synchronize()
    reps = 200
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(reps):
            cp.apply(p)
    graph.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    graph.replay()
    ev[1].record()
    torch.cuda.synchronize()
    apply_s = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
    del graph
    cbytes = 8.0 * n * n + 2 * 16.0 * n
    log(f"[bench] coupling product C p: {apply_s * 1e6:.2f} us per launch, "
        f"{cbytes / apply_s / 1e9:.0f} GB/s")
    # coupled against plain float64 product
    q = torch.ones(n, dtype=torch.complex128, device="cuda")
    for f in (lambda: cp.matvec(p), lambda: plan.matvec(p, q)):
        for _ in range(5):
            f()
    tm = []
    for f in (lambda: cp.matvec(p), lambda: plan.matvec(p, q)):
        ev[0].record()
        for _ in range(100):
            f()
        ev[1].record()
        torch.cuda.synchronize()
        tm.append(ev[0].elapsed_time(ev[1]) * 1e-3 / 100)
    cp.close()
    plan.close()
    log(f"[bench] float64 products: coupled {tm[0] * 1e6:.1f} us, plain {tm[1] * 1e6:.1f} us")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (one whole solve)...")
        v, threads, cdt = cpu_baseline_elastic(E, nodes, tets, V, T, alpha)
        cpu = {"value": v, "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"one whole solve of the same workload ({cdt:.1f} s): dense BEM "
                         f"blocks of the {n} elements, dense K - omega^2 M solve for C, LU "
                         f"of the coupled system (numpy/LAPACK on {threads} threads; the "
                         f"near-field quadrature in one)",
               "affinity_cores": len(os.sched_getaffinity(0)), "cpu_model": cpu_model()}
        log(f"[bench] CPU oracle: {v:.3e} solves/s ({cdt:.1f} s per solve)")
    out = {
        "metric": "elastic-sphere coupled solves/sec (BEM plan + FEM assembly, LU and coupling "
                  "matrix + GMRES to rel resid 1e-5, Sec. 3.1)",
        "value": 1.0 / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "elastic_sphere", "radius": E.radius,
                   "fe_nodes": len(nodes), "fe_unknowns": 3 * len(nodes), "tetrahedra": len(tets),
                   "n_tri": n, "omega": E.omega, "rho_s": E.rho_s, "young": E.young,
                   "poisson": E.poisson, "tol": 1e-5, "fmm_tol": fmm_tol,
                   "alpha": alpha},
        "parts_ms": {"plan": plan_s * 1e3, "coupling": coup_s * 1e3, "gmres": solve_s * 1e3},
        # the coupling build as a whole (assembly, LU, C), live: the
        # algorithmic flops of solving (K - omega^2 M) X = N by LU, 2/3 n^3
        # + 2 n^2 m (factorisation, forward and back substitution), over its
        # measured time (a lower bound for its matrix-core kernels, whose
        # own rates the kernel trace gives)
        "coupling_build": {"ms": coup_s * 1e3, "flop": lu_flop,
                           "TFLOPs": lu_flop / coup_s / 1e12,
                           "frac_fp64_peak": lu_flop / coup_s / PEAK_FP64},
        "gmres_iterations": info["iterations"],
        "adjoint_gmres": {"ms": adj_s * 1e3, "iterations": ainfo["iterations"]},
        "coupling_product": {"us": apply_s * 1e6, "bytes": cbytes,
                             "GBps": cbytes / apply_s / 1e9},
        "matvec_us": {"coupled_f64": tm[0] * 1e6, "plain_f64": tm[1] * 1e6},
        "roofline": {"bound": "hbm", "kernel": "k_real_matvec", "achieved": cbytes / apply_s / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": cbytes / apply_s / HBM_PEAK, "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def m2l_flops(n, nfar, p, cut):
    """Algorithmic FLOPs of n M2L pairs at order p: 8 (p+1)^4 per pair (complex
    multiply-add = 8), the nfar pairs across three boxes reading only the
    (p - cut + 1)^2 input coefficients of degree <= p - cut."""
    pf = max(0, p - cut) if cut > 0 else p
    return 8.0 * ((n - nfar) * (p + 1) ** 4 + nfar * (p + 1) ** 2 * (pf + 1) ** 2)


def rot_m2l_flops(n, nfar, p, cut):
    """Algorithmic FLOPs of n rotation-based M2L pairs at order p: per pair the
    two real rotations (4 (2l+1)^2 per degree l: a real block on a complex
    vector), the coaxial step (8 per complex multiply-add, s^2 per order m,
    s = p + 1 - |m|) and the two phase multiplications (6 per coefficient);
    the nfar pairs across three boxes rotate and translate only the degrees
    <= p - cut of their input."""
    pf = max(0, p - cut) if cut > 0 else p

    def rot(q):
        return sum(4 * (2 * l + 1) ** 2 for l in range(q + 1))

    coax = sum(8 * (p + 1 - abs(m)) ** 2 for m in range(-p, p + 1))
    coax_cut = sum(8 * (p + 1 - abs(m)) * max(0, pf + 1 - abs(m)) for m in range(-p, p + 1))
    nc, kc = (p + 1) ** 2, (pf + 1) ** 2
    full = 2 * rot(p) + coax + 12 * nc
    far = rot(pf) + rot(p) + coax_cut + 6 * kc + 6 * nc
    return float((n - nfar) * full + nfar * far)


def _cpu_points(chunk):
    """Oracle state and adjoint fields, gradients and T_Omega at a few points."""
    from oracle import solve
    geom, k, p, pt, d, obs, amp = _G
    Kh, Sh = solve.represent_blocks(geom, k, chunk)
    inc = np.exp(1j * k * (chunk @ d))
    fs = Kh @ p + inc
    gs = solve.represent_grad(geom, k, chunk, p, None) + (1j * k * inc)[:, None] * d[None, :]
    fa = Kh @ pt + solve.point_source_field(k, chunk, obs, amp)
    ga = solve.represent_grad(geom, k, chunk, pt, None) + solve.point_source_grad(k, chunk, obs, amp)
    return solve.topological_derivative(fs, gs, fa, ga, 1.0, np.inf, 1.0, np.inf, k)


def cpu_baseline_points(V, T, k, p, pt, d, obs, amp, lat, seed, target_s=15.0):
    """The oracle's T_Omega (both fields and gradients by dense sums) on
    sampled lattice points, process-parallel; returns (points/s, cores,
    points, seconds)."""
    import multiprocessing as mp

    from oracle import bem as obem
    cores = min(len(os.sched_getaffinity(0)), 16)
    global _G
    _G = (obem.Geometry(V, T), k, p, pt, d, obs, amp)
    rng = np.random.default_rng(seed)
    pick = lat[rng.permutation(len(lat))]
    t0 = time.perf_counter()
    _cpu_points(pick[:4])
    per_pt = (time.perf_counter() - t0) / 4
    npts = int(max(cores * 4, min(len(lat), target_s * cores / max(per_pt, 1e-6))))
    chunks = np.array_split(pick[:npts], max(1, npts // 4))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        pool.map(_cpu_points, chunks)
    dt = time.perf_counter() - t0
    return npts / dt, cores, npts, dt


def run_topo(args):
    """Topological derivative on the design-domain lattice (the topology
    loop's step 8): state and adjoint fields with their gradients at the
    lattice points by the FMM, then T_Omega.  The state solve (plane wave)
    and the adjoint solve (point sources of intensity 2 conj(p) at the 8
    observation points) run before the timed region."""
    import torch

    import paper_1606_02383_amd as bem
    from workloads import WORKLOADS, unit_directions

    wl = WORKLOADS["sphere81920_k8"]
    V, T = wl.mesh_arrays()
    rng = np.random.default_rng(wl.seed)
    d = unit_directions(rng, 1)[0]
    obs = 3.0 * unit_directions(rng, 8)
    t = np.linspace(-1.25, 1.25, 101)
    X = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    lat = X[np.linalg.norm(X, axis=1) > 1.02]
    plan = bem.Plan(bem.Problem(V, T, wl.k, leaf_cap=64))
    opts = bem.GmresOptions(tol=1e-6, restart=50, mode=1, inner_tol=args.inner_tol)
    p, info = plan.solve(plan.plane_wave_rhs(d), opts=opts)
    pobs = plan.eval_field(p, None, obs, direction=d).cpu().numpy()
    amp = 2.0 * np.conj(pobs)
    pt, info_t = plan.solve(plan.point_source_rhs(obs, amp), opts=opts)
    log(f"[bench] topo: {len(lat)} lattice points; state / adjoint residuals "
        f"{info['resid']:.2e} / {info_t['resid']:.2e}")
    res = {}
    for prec, name in ((bem.BEM_C128, "f64"), (bem.BEM_C64, "f32")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fp = bem.FieldPoints(plan, lat, prec=prec)
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0

        def step():
            fs, gs = fp.eval_field_grad(p, None, direction=d)
            fa, ga = fp.eval_field_grad(pt, None, src=obs, amp=amp)
            return bem.topological_derivative(fs, gs, fa, ga, omega=wl.k)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Tg = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        plan.profile_start()
        step()
        prof = plan.profile_stop()
        res[name] = dict(ms=dt * 1e3, build_s=t_build, stats=fp.stats(), T=Tg.cpu().numpy(),
                         prof=prof)
        log(f"[bench] topo {name}: {dt * 1e3:.2f} ms per T_Omega evaluation "
            f"({len(lat) / dt:.3e} points/s), point set built in {t_build:.2f} s")
        fp.close()
    # the direct sums on a sample of the lattice, for speed and agreement
    pick = np.sort(rng.choice(len(lat), 20000, replace=False))
    sub = lat[pick]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    plan.eval_field_grad(p, None, sub[:256], direction=d)
    ev[0].record()
    fs, gs = plan.eval_field_grad(p, None, sub, direction=d)
    fa, ga = plan.eval_field_grad(pt, None, sub, src=obs, amp=amp)
    Td = bem.topological_derivative(fs, gs, fa, ga, omega=wl.k)
    ev[1].record()
    torch.cuda.synchronize()
    direct_ms = ev[0].elapsed_time(ev[1]) * len(lat) / len(sub)
    Td = Td.cpu().numpy()
    err = {n: float(np.linalg.norm(res[n]["T"][pick] - Td) / np.linalg.norm(Td)) for n in res}
    log(f"[bench] topo direct sums: {direct_ms:.1f} ms for the lattice (from 20000 points); "
        f"T_Omega rel. difference FMM vs direct: f64 {err['f64']:.2e}, f32 {err['f32']:.2e}")
    # roofline: the leaf-level M2L into the point boxes (float64), timed by
    # HIP events on the stream in the profiled step (two evaluations)
    r64 = res["f64"]
    st = r64["stats"]
    L = st["levels"]
    ms_leaf, calls_leaf = r64["prof"].get(("m2l_leaf", "f64", "fwd"), (0.0, 0))
    # algorithmic FLOPs of the algorithm the leaf level runs (rotation-based
    # where the problem's float64 leaf M2L is, else dense operators)
    rot_leaf = bool(st["m2l_rot"][L])
    dense = m2l_flops(st["n_m2l"][L], st["n_m2l_far"][L], st["order"][L], st["far_cut"])
    flops = (rot_m2l_flops(st["n_m2l"][L], st["n_m2l_far"][L], st["order"][L], st["far_cut"])
             if rot_leaf else dense)
    per_ms = ms_leaf / max(1, calls_leaf)
    ach = flops / (per_ms / 1e3) if per_ms > 0 else 0.0
    stages = {f"{k_[0]}_{k_[1]}": round(v[0] / v[1], 4) for k_, v in r64["prof"].items()}
    kern = ("k_rot_m2l<double,256,false> (rotation-based, results added atomically)" if rot_leaf
            else "k_grouped_gemm<double,*,false,1>")
    roofline = {"kernel": f"{kern} (leaf-level M2L into the point boxes, float64)",
                "bound": "mfma", "achieved": round(ach / 1e12, 3),
                "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64, 4),
                "traffic": None, "flops_per_launch": flops, "dense_equivalent_flops": dense,
                "avg_launch_ms": round(per_ms, 5), "launches": calls_leaf,
                "rotation_based_levels": [l for l in range(2, L + 1) if st["m2l_rot"][l]]}
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (sampled lattice points)...")
        v, cores, npts, cdt = cpu_baseline_points(V, T, wl.k, p.cpu().numpy(), pt.cpu().numpy(),
                                                  d, obs, amp, lat, wl.seed)
        cpu = {"value": v, "unit": "points/s", "cores": cores, "kind": "oracle",
               "sample": f"T_Omega at {npts} of {len(lat)} lattice points (both fields and "
                         f"gradients by dense numpy sums over all elements, {cores} processes, "
                         f"{cdt:.1f} s)",
               "affinity_cores": len(os.sched_getaffinity(0)), "cpu_model": cpu_model()}
        log(f"[bench] CPU oracle: {v:.3e} points/s on {cores} cores")
    out = {
        "metric": "T_Omega lattice points/sec (state and adjoint field + gradient by FMM at "
                  "the 101^3 design-domain lattice points outside the sphere N=81920, k=8)",
        "value": len(lat) / (r64["ms"] / 1e3), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "topo_sphere81920_k8", "n_tri": len(T), "k": wl.k,
                   "lattice": "101^3 on [-1.25, 1.25]^3, points with |x| > 1.02",
                   "n_points": len(lat), "material": "sound-hard limit",
                   "objective": "sum |p|^2 over 8 points on the radius-3 sphere"},
        "f32": {"ms_per_step": res["f32"]["ms"], "points_per_s": len(lat) / (res["f32"]["ms"] / 1e3),
                "T_rel_diff_vs_direct": err["f32"],
                "stage_ms_per_call": {f"{k_[0]}_{k_[1]}": round(v[0] / v[1], 4)
                                      for k_, v in res["f32"]["prof"].items()}},
        "T_rel_diff_vs_direct": err["f64"],
        "direct_sum_ms": direct_ms,
        "point_set_build_s": {"f64": r64["build_s"], "f32": res["f32"]["build_s"]},
        "point_tree": {"n_box": st["n_box"][2:], "n_m2l": st["n_m2l"][2:],
                       "order": st["order"][2:], "n_leaf": st["n_leaf"],
                       "n_near_pairs": st["n_near_pairs"]},
        "stage_ms_per_call": stages,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# Algorithmic work of the float32 near field per (target, source element)
# pair for the rigid products timed here (alpha = i/k, q = 0), counted on the
# pair kernel's expression (add, subtract, multiply = 1 FLOP, fused
# multiply-add = 2; 1/sqrt, sin and cos counted apart): per rule point
# r = x - y (3), |r|^2 (5), |r| (1), k|r| (1), G = e^{ik|r|}/|r| (2), 1/|r|^2
# (1), r.n_x (5), k/|r| and alpha k/|r| (2), the two products of the
# double-normal term (2), the p coefficient's real (4) and imaginary (7)
# parts and its complex multiply-add into the element sum (8): 41; per
# element n_x.n_y (5), r.n_y (6), alpha n_x.n_y (1) and the density's complex
# multiply-add (8) less the first point's start of the sum (2): 18.
# Element pair: 3 x 41 + 18 = 141 FLOPs and 9 transcendentals.  Each near
# correction adds one complex multiply-add (8).
P2P_FLOPS_PER_PAIR = 141
P2P_TRANS_PER_PAIR = 9
P2P_FLOPS_PER_CORRECTION = 8
PEAK_VEC_NONPACKED = 78.6e12   # float32 vector FMA rate without packed instructions


def p2p_roofline(st, prof, alone):
    """Algorithmic FLOP/s of the float32 near field, in the product (stage
    profile, sharing the GPU with the far field) and alone (serial profile)."""
    flops = (st["n_p2p_pairs"] * P2P_FLOPS_PER_PAIR
             + st["n_near"] * P2P_FLOPS_PER_CORRECTION)
    out = {"kernel": "k_p2p<float,true,true> (near field, float32, q = 0)", "bound": "alu",
           "flops_per_element_pair": P2P_FLOPS_PER_PAIR,
           "transcendentals_per_element_pair": P2P_TRANS_PER_PAIR,
           "element_pairs": st["n_p2p_pairs"], "near_corrections": st["n_near"],
           "flops_per_launch": flops, "peak": PEAK_VEC_NONPACKED / 1e12, "unit": "TFLOP/s"}
    for name, pr in (("in_product", prof), ("alone", alone)):
        ms, calls = pr.get(("p2p", "f32", "fwd"), (0.0, 0))
        if calls:
            t = ms / calls / 1e3
            out[f"{name}_ms"] = round(t * 1e3, 5)
            out[f"achieved_{name}"] = round(flops / t / 1e12, 3)
            out[f"frac_{name}"] = round(flops / t / PEAK_VEC_NONPACKED, 4)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere81920_k8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--inner-tol", type=float, default=1e-3)
    ap.add_argument("--counters", action="store_true",
                    help="short run for hardware-counter passes: 3 float32 and 3 float64 "
                         "products, then one elementwise kernel over 512 MiB in / 512 MiB out "
                         "(the byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "path is a design, not part of this build", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch32":
        run_batch(args)
        return
    if args.workload == "grad_cube49152_k6":
        run_grad(args)
        return
    if args.workload == "topo_sphere81920_k8":
        run_topo(args)
        return
    if args.workload == "elastic_sphere":
        run_elastic(args)
        return
    import torch

    import paper_1606_02383_amd as bem
    from workloads import WORKLOADS, unit_directions

    wl = WORKLOADS[args.workload]
    V, T = wl.mesh_arrays()
    rng = np.random.default_rng(wl.seed)
    d = unit_directions(rng, 1)[0]
    log(f"[bench] workload {wl.name}: n_tri={len(T)} k={wl.k}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = bem.Plan(bem.Problem(V, T, wl.k, leaf_cap=64))
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    st = plan.stats()
    log(f"[bench] plan built in {t_plan:.2f} s; leaf level {st['leaf_level']}, "
        f"orders f64 {st['order64'][2:]} f32 {st['order32'][2:]}, m2l pairs {st['n_m2l'][2:]}, "
        f"P2P pairs {st['n_p2p_pairs']}, schedule f64/f32 {st['schedule']}, "
        f"P2P grid {st['p2p_grid']}, leaf M2L grid {st['m2l_grid']}, "
        f"direct depth {st['direct_depth']}, far cut {st['far_cut']}")
    b = plan.plane_wave_rhs(d)
    if args.counters:
        for prec in (1, 0):
            for _ in range(3):
                plan.matvec(b, prec=prec)
        x = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        log("[bench] counters run done")
        return
    opts64 = bem.GmresOptions(tol=wl.tol, restart=50, mode=0)
    optsir = bem.GmresOptions(tol=wl.tol, restart=50, mode=1, inner_tol=args.inner_tol)

    # float64 reference solve (once warm-up, once timed)
    plan.solve(b, opts=opts64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x64, info64 = plan.solve(b, opts=opts64)
    torch.cuda.synchronize()
    t64_solve = time.perf_counter() - t0
    log(f"[bench] f64 GMRES: {info64['matvec64']} matvecs, resid {info64['resid']:.2e}, "
        f"{t64_solve * 1e3:.1f} ms")

    # raw matvec throughput: 3 warm-ups, then the median of 20 products, each
    # bracketed by HIP events on the caller's stream (the product's side
    # streams join it before the product ends)
    p = torch.randn(len(T), dtype=torch.complex128, device="cuda")
    rates = {}
    for prec, name in ((0, "f64"), (1, "f32")):
        for _ in range(3):
            plan.matvec(p, prec=prec)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(20)]
        for e0, e1 in ev:
            e0.record()
            plan.matvec(p, prec=prec)
            e1.record()
        torch.cuda.synchronize()
        med = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
        rates[name] = 1e3 / med
        log(f"[bench] {name} matvec: {med:.3f} ms (median of 20)")

    # timed mixed-precision solves
    for _ in range(args.warmup):
        plan.solve(b, opts=optsir)
    torch.cuda.synchronize()
    # the dominant kernel (leaf-level float32 M2L) is timed inside the timed
    # region by HIP events attached to its launches (nothing is recorded
    # between kernels, so the schedule of the solves is unchanged)
    plan.profile_start(leaf_m2l_only=True)
    t0 = time.perf_counter()
    infos = []
    for s_ in range(args.steps):
        x, info = plan.solve(b, opts=optsir)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    leaf_prof = plan.profile_stop()
    ms_step = dt / args.steps * 1e3
    info = infos[-1]
    sol_err = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
    log(f"[bench] IR solve: {ms_step:.1f} ms/step, mv32 {info['matvec32']} mv64 "
        f"{info['matvec64']}, resid {info['resid']:.2e}, |x - x64|/|x64| {sol_err:.2e}")
    value = info64["matvec64"] / (ms_step / 1e3)

    # stage profile of one mixed-precision solve (HIP events on the stream)
    plan.profile_start()
    plan.solve(b, opts=optsir)
    prof = plan.profile_stop()
    stages = {f"{k[0]}_{k[1]}_{k[2]}": round(v[0] / v[1], 4) for k, v in prof.items()}
    # every stage alone on the GPU: products with q = 0 (as in the rigid
    # solves) on one stream, one stage after another
    plan.profile_start(serial=True)
    for prec in (1, 0):
        for _ in range(3):
            plan.matvec(p, prec=prec)
    alone = plan.profile_stop()
    stages_alone = {f"{k[0]}_{k[1]}_{k[2]}": round(v[0] / v[1], 4) for k, v in alone.items()}
    # dominant kernel: the leaf-level float32 M2L GEMM (one launch per
    # product); algorithmic flops per launch = 8 (p_L + 1)^4 per M2L pair,
    # 8 (p_L + 1)^2 (p_L - far_cut + 1)^2 for the pairs across three boxes
    L = st["leaf_level"]
    leaf_ms, leaf_calls = leaf_prof.get(("m2l_leaf", "f32", "fwd"), (0.0, 0))
    fc32 = st["far_cut"][1]
    flops_leaf = m2l_flops(st["n_m2l"][L], st["n_m2l_far"][L], st["order32"][L], fc32)
    per_launch_ms = leaf_ms / max(1, leaf_calls)
    achieved = flops_leaf / (per_launch_ms / 1e3) if per_launch_ms > 0 else 0.0
    coarse_ms, coarse_calls = prof.get(("m2l", "f32", "fwd"), (0.0, 0))
    flops_coarse = sum(m2l_flops(st["n_m2l"][l], st["n_m2l_far"][l], st["order32"][l], fc32)
                       for l in range(2, L))
    coarse_launch_ms = coarse_ms / max(1, coarse_calls)
    roofline = {"kernel": f"k_grouped_gemm<float,{st['m2l_tile32'][L]},false,0> "
                          f"(leaf-level M2L, float32)", "bound": "mfma",
                "achieved": round(achieved / 1e12, 3), "peak": PEAK_FP32_MFMA / 1e12,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA, 4),
                "traffic": measured_traffic(),
                "flops_per_launch": flops_leaf, "avg_launch_ms": round(per_launch_ms, 5),
                "launches": leaf_calls,
                "coarse_levels_m2l": {"flops_per_launch": flops_coarse,
                                      "avg_launch_ms": round(coarse_launch_ms, 5),
                                      "tflops": round(flops_coarse / max(coarse_launch_ms, 1e-9)
                                                      / 1e9, 3)},
                "alone_ms": round(alone.get(("m2l_leaf", "f32", "fwd"), (0.0, 1))[0]
                                  / max(1, alone.get(("m2l_leaf", "f32", "fwd"), (0.0, 1))[1]),
                                  5),
                "p2p": p2p_roofline(st, prof, alone)}

    # float64 leaf-level M2L (the refinement's float64 products; rotation-based
    # where the plan's tuner found it faster): algorithmic FLOPs of the
    # algorithm run, and those of the same translations by dense operators
    rot64 = st["m2l_rot64"]
    fc64 = st["far_cut"][0]
    dense64 = m2l_flops(st["n_m2l"][L], st["n_m2l_far"][L], st["order64"][L], fc64)
    flops64 = (rot_m2l_flops(st["n_m2l"][L], st["n_m2l_far"][L], st["order64"][L], fc64)
               if rot64[L] else dense64)
    f64_ms, f64_calls = prof.get(("m2l_leaf", "f64", "fwd"), (0.0, 0))
    f64_alone_ms, f64_alone_calls = alone.get(("m2l_leaf", "f64", "fwd"), (0.0, 0))
    f64_launch = f64_ms / max(1, f64_calls)
    f64_alone = f64_alone_ms / max(1, f64_alone_calls)
    m2l64 = {"kernel": ("k_rot_m2l<double,256,false> (rotation-based)" if rot64[L]
                        else "k_grouped_gemm<double,...,false,0> (dense)"),
             "rotation_based_levels": [l for l in range(2, L + 1) if rot64[l]],
             "order": st["order64"][L], "far_cut": fc64,
             "flops_per_launch": flops64, "dense_equivalent_flops": dense64,
             "avg_launch_ms": round(f64_launch, 5), "alone_ms": round(f64_alone, 5),
             "tflops_alone": round(flops64 / max(f64_alone, 1e-9) / 1e9, 3),
             "frac_alone": round(flops64 / max(f64_alone, 1e-9) / 1e9 / (PEAK_FP64 / 1e12), 4),
             "peak_tflops": PEAK_FP64 / 1e12}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (sampled rows)...")
        v, cores, nrows, cdt = cpu_baseline(V, T, wl.k, wl.seed)
        cpu = {"value": v, "unit": "matvecs/s", "cores": cores, "kind": "oracle",
               "sample": f"{nrows} of {len(T)} rows of one float64 dense matrix-free matvec "
                         f"(numpy, {cores} processes, {cdt:.1f} s), scaled to whole matvecs",
               "affinity_cores": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count(),
               "cpu_model": cpu_model()}
        log(f"[bench] CPU oracle: {v:.3e} matvecs/s on {cores} cores")

    out = {
        "metric": "FMM-BEM matvecs/sec at N=81920,k=8 (FP32+refine vs FP64, rel err 1e-6)",
        "value": value, "unit": "matvecs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64+c128",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_tri": len(T), "k": wl.k, "alpha": "i/k",
                   "rhs": "plane wave, seeded direction", "tol": wl.tol,
                   "solver": "GMRES(50), float32 inner / float64 refinement",
                   "inner_tol": args.inner_tol, "leaf_level": L, "schedule": st["schedule"],
                   "order32": st["order32"][2:], "order64": st["order64"][2:],
                   "far_cut": st["far_cut"], "m2l_rotation_levels_f64": st["m2l_rot64"][2:],
                   "m2l_rotation_levels_f32": st["m2l_rot32"][2:]},
        "f64_gmres": {"matvecs": info64["matvec64"], "ms": t64_solve * 1e3,
                      "matvecs_per_s": info64["matvec64"] / t64_solve},
        "ir_solve": {"matvec32": info["matvec32"], "matvec64": info["matvec64"],
                     "resid": info["resid"], "rel_diff_vs_f64_solution": sol_err},
        "matvec_per_s": {"f64": rates["f64"], "f32": rates["f32"]},
        "sampled_error": {"f64_white_noise": st["fmm_err64"], "f64_plane_wave": st["fmm_err64_smooth"],
                          "f32_white_noise": st["fmm_err32"], "f32_plane_wave": st["fmm_err32_smooth"],
                          "rows": 128, "reference": "rows summed directly in float64"},
        "plan_build_s": t_plan,
        "stage_ms_per_call": stages,
        "stage_ms_alone": stages_alone,
        "roofline": roofline,
        "m2l_f64_leaf": m2l64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
