"""Benchmark of the state-vector ADAPT-VQE hot path on one MI355X.

One step = one pass of the whole hot path over the resident synthetic state:
sigma = H psi (FP64), the energy <psi|sigma>, the full pool-gradient sweep
g_k = 2 <sigma|A_k psi>, and one exponentiated-operator rotation of psi.
Prints one JSON line.  The headline value is the H psi rate in GB/s under the
gather model (every structural nonzero's source amplitude read once, the
output written once, plus the Pauli table), measured with HIP events on the
stream the kernels run on.  The oracle leg times the plain CPU oracle on a
bounded sample of output rows of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_VECTOR_TFLOPS = 78.6    # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz; the FP64 matrix peak is the same


def model(M, na, nb, T, pool):
    """Closed-form sizes of the workload (per H psi / per sweep)."""
    da, db = math.comb(M, na), math.comb(M, nb)
    dim = da * db
    sa, sb = na * (M - na), nb * (M - nb)
    dda = math.comb(na, 2) * math.comb(M - na, 2)
    ddb = math.comb(nb, 2) * math.comb(M - nb, 2)
    conn = 1 + sa + sb + dda + ddb + sa * sb
    nnz = dim * conn
    pairs = (nnz - dim) // 2
    return dict(dim=dim, da=da, db=db, conn=conn, nnz=nnz, pairs=pairs, sa=sa, sb=sb,
                dda=dda, ddb=ddb, T=T, pool=pool, M=M, na=na, nb=nb)


def hpsi_gather_bytes(m, S=8):
    return (m["nnz"] + m["dim"]) * S + 16 * m["T"]


def kernel_flops(name, m):
    """Algorithmic flops of one launch: 2 per structural nonzero (FMA) the
    kernel handles, 2 per (target, source) product of the transition-value
    pass, 2 M N K for the Gram GEMMs, 4 per pair for the pair kernel."""
    dim, sa, sb = m["dim"], m["sa"], m["sb"]
    if name == "k_mixed":
        return 2.0 * dim * (sa * sb + sa + sb + 1), "alu"
    if name == "k_mixed_m":  # the same products on the FP64 matrix cores
        return 2.0 * dim * (sa * sb + sa + sb + 1), "mfma"
    if name == "k_ss_apply":  # mean of the alpha- and the beta-row launch
        return 2.0 * dim * (1 + (sa + m["dda"] + sb + m["ddb"]) / 2), "alu"
    if name in ("k_tdens", "k_tdens_rows"):
        return 2.0 * dim * (sa + sb * (sa + 1)), "alu"
    if name == "k_tdens_m":  # the same products on the FP64 matrix cores
        return 2.0 * dim * (sa + sb * (sa + 1)), "mfma"
    if name in ("k_core_gram_a", "k_core_gram_b"):
        # 2 flops per (core, slot i, slot j, column): the S x S block of every
        # (N-2)-electron core over the other spin's strings
        M = m["M"]
        N = m["na"] if name.endswith("_a") else m["nb"]
        K = m["db"] if name.endswith("_a") else m["da"]
        S = math.comb(M - N + 2, 2)
        return 2.0 * math.comb(M, N - 2) * S * S * K, "mfma"
    if name == "k_pool_grad":
        return 4.0 * m["pairs"], "alu"
    return 2.0 * m["nnz"], "alu"


# LDS: 128 bytes per clock per CU, 256 CUs at 2.4 GHz
LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12


def roofline(name, ms, m):
    flops, bound = kernel_flops(name, m)
    achieved = flops / (ms * 1e-3) / 1e12
    out = {"bound": bound, "kernel": name, "achieved": round(achieved, 3), "peak": FP64_VECTOR_TFLOPS,
           "unit": "TFLOP/s", "frac": round(achieved / FP64_VECTOR_TFLOPS, 4), "traffic": None,
           "ms_per_launch": round(ms, 3)}
    # the LDS-staged product kernels: algorithmic LDS read bytes per launch
    # (two 8-byte reads per mixed-pass product: coefficient and amplitude;
    # one per transition-value product) against the chip's LDS bandwidth
    per_product = {"k_mixed": 16.0, "k_tdens_rows": 8.0}.get(name)
    if per_product is not None:
        lds = flops / 2.0 * per_product / (ms * 1e-3) / 1e12
        out["lds"] = {"achieved": round(lds, 2), "peak": round(LDS_PEAK_TBS, 1), "unit": "TB/s",
                      "frac": round(lds / LDS_PEAK_TBS, 4)}
    return out


# source file of each kernel whose counters are committed
KERNEL_SOURCES = {"k_mixed": "hamiltonian.hip", "k_mixed_m": "hamiltonian.hip", "k_ss_apply": "hamiltonian.hip", "k_transpose": "hamiltonian.hip",
                  "k_ss_core": "hamiltonian.hip", "k_ss_apply_sparse": "hamiltonian.hip",
                  "k_ssg_compact": "hamiltonian.hip", "k_tdens_rows": "sweep.hip", "k_tdens_m": "sweep.hip",
                  "k_tm_final": "sweep.hip", "k_tdens_rows_final": "sweep.hip",
                  "k_gram_grad": "sweep.hip", "k_core_gram_a": "core_gram.hip", "k_core_gram_b": "core_gram.hip",
                  "k_gram_transpose": "core_gram.hip", "k_rotate": "pool.hip", "k_dot_partial_f64": "sector.hip"}


def source_digest(kernel=None):
    """Digest of a kernel's source file and the shared header (all sources
    when kernel is None or unknown)."""
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2604_01176_amd", "csrc")
    if kernel in KERNEL_SOURCES:
        files = [os.path.join(csrc, KERNEL_SOURCES[kernel]), os.path.join(csrc, "hyp_internal.h")]
    else:
        files = sorted(glob.glob(os.path.join(csrc, "*")))
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when there is none or the kernel's source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    k = t.get("kernels", {}).get(kernel)
    if k is None or k.get("source_digest") != source_digest(kernel):
        return None
    return k.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="h16_32q")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time budget of the oracle leg (0 disables it)")
    ap.add_argument("--no-sweep", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the near-Hartree-Fock and assembly measurements (profiling runs: keeps every "
                         "launch of the step's kernels at the benchmark state)")
    ap.add_argument("--fp32-study", type=int, default=0, metavar="ITERS",
                    help="FP32-storage vs FP64 error study over ITERS ADAPT iterations (JSON lines)")
    ap.add_argument("--adapt-compare", type=int, default=0, metavar="ITERS",
                    help="screened FP32 vs plain FP64 ADAPT iterations on the workload (JSON lines)")
    ap.add_argument("--adapt-early", type=int, default=0, metavar="ITERS",
                    help="plain FP64 ADAPT from Hartree-Fock, support skipping on, then off")
    ap.add_argument("--skip-only", action="store_true",
                    help="with --adapt-early: only the run with support skipping (longer trajectories)")
    ap.add_argument("--csr", action="store_true",
                    help="materialised CSR SpMV against the matrix-free product (24- and 28-qubit workloads)")
    ap.add_argument("--graph", action="store_true",
                    help="inner-optimiser evaluation (state prep + H psi + E + adjoint gradient): captured graph vs eager")
    ap.add_argument("--cpu-study", action="store_true",
                    help="the CPU oracle timed on this host at 1 thread and all threads (H psi, sweep, ADAPT)")
    ap.add_argument("--batch", action="store_true",
                    help="full pool-gradient sweeps of the eight uneven batch instances: one persistent batched "
                         "launch (autotuned tile) against per-instance sweeps (JSON line)")
    ap.add_argument("--shadow", action="store_true",
                    help="with --adapt-compare: also judge every screened iteration by a full sweep on its own "
                         "state (diagnostic; the extra sweeps are not in the screened timings)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (hardware-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the beta-row-partitioned design is described in the design notes, not implemented).",
              file=sys.stderr)
        sys.exit(2)

    if args.cpu_study:  # host only: no GPU needed
        cpu_study()
        return

    import numpy as np
    import torch
    import synth
    import paper_2604_01176_amd as hyp

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 8, "bytes_written": n * 8, "copies": 3}))
        return
    if args.batch:
        batch_bench()
        return
    if args.csr:
        csr_bench()
        return
    if args.graph:
        graph_bench()
        return

    w = synth.WORKLOADS[args.workload]
    if args.fp32_study:
        fp32_study(w, args.fp32_study)
        return
    if args.adapt_compare:
        adapt_compare(w, args.adapt_compare, args.shadow)
        return
    if args.adapt_early:
        adapt_early(w, args.adapt_early, args.skip_only)
        return
    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    t0 = time.time()
    x, z, c, h_int, g_int = synth.hamiltonian(w)
    cre, ann, cls = synth.canonical_pool(M)
    m = model(M, na, nb, len(c), len(cre))
    print(f"[bench] {w.name}: dim {m['dim']}, {m['T']} Pauli terms, pool {m['pool']}, "
          f"inputs built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    assert H.structured
    psi_h = synth.random_state(S.dim, 7)
    psi = torch.from_numpy(psi_h).cuda()
    sig = torch.empty_like(psi)
    ops = hyp.exc_tensor(cre, ann)
    grad = torch.empty(len(cre), dtype=torch.float64, device="cuda")
    e_dev = torch.empty(1, dtype=torch.float64, device="cuda")
    k_rot = int(np.nonzero(cls == 4)[0][0])

    def step():
        hyp.hyp_apply_h(H, psi, sig)
        hyp.hyp_expectation(S, psi, sig, e_dev)
        if not args.no_sweep:
            hyp.hyp_pool_gradients(S, ops, psi, sig, grad)
        hyp.hyp_apply_excitation(S, int(cre[k_rot]), int(ann[k_rot]), 1e-3, psi)

    # the library's tile autotuner picks the mixed pass's workgroup width on
    # this Hamiltonian (it overwrites sig, which step() recomputes)
    hpsi_threads, tune_ms = H.tune(psi, reps=1)
    print(f"[bench] H psi autotune: {hpsi_threads} threads per workgroup ({tune_ms:.1f} ms)",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    hyp.profile_reset()
    hyp.profile_enable(True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for i in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    hyp.profile_enable(False)
    step_ms = ev0.elapsed_time(ev1) / args.steps
    prof = hyp.profile_read()
    g_prev_step = grad.cpu().numpy()  # the last step's sweep, one rotation before the current state
    print(f"[bench] timed {args.steps} steps: {step_ms:.2f} ms/step", file=sys.stderr, flush=True)
    for k_, (ms, n) in sorted(prof.items(), key=lambda kv: -kv[1][0]):
        print(f"[bench]   {k_:20s} {ms / max(n, 1):10.3f} ms/launch x {n}", file=sys.stderr)

    # FP32 storage (FP64 accumulation) H psi on the same state, tuned for FP32
    psi32 = psi.float()
    sig32 = torch.empty_like(psi32)
    threads32, _ = H.tune(psi32, reps=1)
    hyp.hyp_apply_h(H, psi32, sig32)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(2):
        hyp.hyp_apply_h(H, psi32, sig32)
    e1.record()
    torch.cuda.synchronize()
    hpsi32_ms = e0.elapsed_time(e1) / 2
    del psi32, sig32
    print(f"[bench] H psi FP32 storage: {hpsi32_ms:.1f} ms ({threads32} threads)", file=sys.stderr, flush=True)

    # support skipping near Hartree-Fock (an early-ADAPT state: HF and 24
    # determinants one pool excitation away), H psi and the full sweep,
    # skipping on against off
    sup, asm = None, None
    if not args.no_extras:
        sup, asm = extras(hyp, torch, np, synth, S, H, ops, grad, w, M, na, nb)

    # H psi wall time on the caller's stream (the same-spin pass overlaps the
    # mixed pass on a side stream, so summed kernel times would overcount)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        hyp.hyp_apply_h(H, psi, sig)
    e1.record()
    torch.cuda.synchronize()
    hpsi_ms = e0.elapsed_time(e1) / 3
    hpsi_bytes = hpsi_gather_bytes(m)
    value = hpsi_bytes / (hpsi_ms * 1e-3) / 1e9
    sweep_kernels = ("k_pool_grad", "k_sum_chunks", "k_tdens", "k_tdens_reduce_ab", "k_tdens_reduce_a",
                     "k_tdens_final", "k_tdens_rows", "k_tdens_rows_final", "k_eb_rows", "k_gram_grad",
                     "k_tdens_grad", "k_core_gram_a", "k_core_gram_b", "k_gram_transpose", "k_gram_widen",
                     "k_zero_u32", "k_support", "k_list_nz", "k_rows_compact", "k_tdens_m", "k_tm_final")
    sweep_ms = sum(prof.get(k, (0.0, 0))[0] for k in sweep_kernels) / args.steps

    # the learned screen's gradient phase on the same state (network trained
    # in-run on the 8-, 16- and 24-qubit workloads)
    screened = None
    if not args.no_extras:
        screened = screened_leg(hyp, torch, np, synth, S, H, psi, g_prev_step, cre, ann, cls, h_int, g_int,
                                sweep_ms)
        print(f"[bench] screened: {json.dumps(screened)}", file=sys.stderr, flush=True)

    # dominant kernel of the step and its roofline
    dom = max(prof.items(), key=lambda kv: kv[1][0])[0]
    dom_ms = prof[dom][0] / prof[dom][1]
    roof = roofline(dom, dom_ms, m)
    roof["traffic"] = measured_traffic(w.name, dom)
    # H psi's measured HBM bytes (committed counter table) over its time: the
    # DRAM-counter fraction of the HBM peak (null when a kernel's table entry
    # is missing or stale)
    # (bytes per launch of each H psi kernel x its launches per product; the
    # same-spin pass runs in column bands, several launches per product)
    hk = [k for k in ("k_mixed", "k_mixed_m", "k_ss_core", "k_ss_apply", "k_ss_apply_sparse", "k_transpose") if k in prof]
    hb = {k: measured_traffic(w.name, k) for k in hk}
    hpsi_hbm = None
    if hk and all(v is not None for v in hb.values()):
        bytes_per_hpsi = sum(hb[k] * prof[k][1] / args.steps for k in hk)
        hpsi_hbm = {"bytes": round(bytes_per_hpsi), "gbs": round(bytes_per_hpsi / (hpsi_ms * 1e-3) / 1e9, 1),
                    "frac": round(bytes_per_hpsi / (hpsi_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        rng = np.random.default_rng(0)
        # calibrate on growing samples until one takes >= 1 s, then size the
        # timed sample to about cpu_seconds of oracle work
        n_try, dt = 256, 0.0
        while True:
            t = time.time()
            oracle.apply_h(M, na, nb, x, z, c, psi_h, out_idx=rng.integers(0, S.dim, n_try))
            dt = time.time() - t
            if dt >= 1.0 or n_try >= 4_000_000:
                break
            n_try *= 4
        n_rows = int(max(256, min(20_000_000, n_try * args.cpu_seconds / max(dt, 1e-6))))
        idx = rng.integers(0, S.dim, n_rows)
        t = time.time()
        oracle.apply_h(M, na, nb, x, z, c, psi_h, out_idx=idx)
        dt = time.time() - t
        row_bytes = (m["conn"] + 1) * 8
        if asm is not None:
            from oracle import jw
            t_j = time.time()
            jw.jw_pauli_list(*synth.integrals(w.n_orb, w.seed))
            asm["oracle_s"] = round(time.time() - t_j, 2)
        cpu = {"value": round(n_rows * row_bytes / dt / 1e9, 4), "unit": "GB/s",
               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
               "kind": "oracle",
               "sample": f"{n_rows} random output rows of H psi ({dt:.1f} s), gather-model bytes"}

    out = {
        "metric": "H psi effective GB/s (gather-model bytes / time; DRAM-counter fraction in hpsi_hbm_measured) "
                  "+ pool-grad evals/s, plain vs screened",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {2 * M} qubits, sector ({na},{nb}), dim {m['dim']}, "
                               f"{m['T']} Pauli terms, pool {m['pool']}",
                   "parallelism": "1 GPU"},
        "hpsi_ms": round(hpsi_ms, 3), "hpsi_threads": int(hpsi_threads),
        "hpsi_fp32_ms": round(hpsi32_ms, 3), "hpsi_fp32_threads": int(threads32),
        "hpsi_frac_hbm_gather_model": round(value / HBM_PEAK_GBS, 4),
        "hpsi_hbm_measured": hpsi_hbm,
        "pool_grad_evals_per_s": round(m["pool"] / (sweep_ms * 1e-3), 1) if sweep_ms > 0 else None,
        "sweep_ms": round(sweep_ms, 3),
        "screened": screened,
        "support_skip_near_hf": sup,
        "pauli_assembly": asm,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def train_screen(hyp, np, synth, scr):
    """The screen's network trained in-run with the library's kernels on
    exact sweeps of plain ADAPT runs on the 8-, 16- and 24-qubit workloads
    (floored residual targets, 16 epochs of Adam)."""
    t0 = time.time()
    Xs, ts = [], []
    for k, (name, iters) in enumerate((("h4_8q", 8), ("h8_16q", 12), ("h12_24q", 6))):
        v = synth.WORKLOADS[name]
        x, z, c, h, g = synth.hamiltonian(v)
        cre, ann, cls = synth.canonical_pool(v.n_orb)
        S = hyp.Sector(v.n_orb, v.n_alpha, v.n_beta)
        H = hyp.Hamiltonian(S, x, z, c)
        A = hyp.Adapt(H, cre, ann, max_iter=iters + 1)
        stat, qidx = scr.static_features(v.n_orb, cre, ann, cls, h, g)
        X, t = scr.collect_rows(A, scr.FeatureState(S, stat, qidx), iters, seed=k)
        Xs.append(X)
        ts.append(t)
        del A, H, S
    X = np.concatenate(Xs)
    t = np.concatenate(ts)
    net = scr.MLP(synth.mlp_init(0), 1 << 16)
    losses = scr.train(net, X, t, epochs=16, batch=1024, lr=1e-3)
    return net, {"rows": int(X.shape[0]), "loss_first_last": [round(losses[0], 4), round(losses[-1], 4)],
                 "train_s": round(time.time() - t0, 1)}


def screened_leg(hyp, torch, np, synth, S, H, psi, psi_prev_grad, cre, ann, cls, h, g, sweep_ms,
                 K=512, audit=256, judge_every=10, reps=3):
    """The screened gradient phase on the benchmark state, as the screened
    ADAPT iteration runs it: occupations + feature rows + base scores, MLP
    scores, ranking and candidate choice (top K, the band below it, a
    uniform audit), exact gradients of the K + audit candidates, the
    fallback test; the judge's full sweep every judge_every-th iteration is
    amortised, and a fallback would add a full sweep.  g_prev is the full
    sweep of the previous step's state (one rotation earlier).  FP64 and FP32
    storage.  Evaluations/s = pool size / that time (the plain rate is pool
    size / full-sweep time)."""
    from paper_2604_01176_amd import screen as scr
    net, train = train_screen(hyp, np, synth, scr)
    M = S.n_orb
    n = len(cre)
    stat, qidx = scr.static_features(M, cre, ann, cls, h, g)
    out = {"K": K, "audit": audit, "judge_every": judge_every, "training": train,
           "g_prev": "full sweep of the previous step's state"}
    sig = torch.empty_like(psi)
    hyp.hyp_apply_h(H, psi, sig)
    g_now = hyp.hyp_pool_gradients(S, hyp.exc_tensor(cre, ann), psi, sig).cpu().numpy()
    kstar = int(np.argmax(np.abs(g_now)))
    for tag, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        p = psi.to(dt)
        sg = torch.empty_like(p)
        hyp.hyp_apply_h(H, p, sg)
        fs = scr.FeatureState(S, stat, qidx)
        fs.update(psi_prev_grad)
        times = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X = fs.features(p)
            y = net.forward(X)
            order = net.rank(y, fs.base).cpu().numpy()
            t1 = time.perf_counter()
            r_top, r_band, r_aud = scr.candidate_ranks(n, K, audit, 42, r)
            top = order[r_top]
            outside = order[np.concatenate([r_band, r_aud])]
            cand = np.concatenate([top, outside]).astype(np.int64)
            gc = hyp.hyp_pool_gradients(S, hyp.exc_tensor(cre[cand], ann[cand]), p, sg).cpu().numpy()
            gt, go = np.abs(gc[:top.size]), np.abs(gc[top.size:])
            fallback = bool(go.size and go.max() >= scr.RHO * gt.max())
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if r > 0:  # the first pass builds scratch and tables
                times.append(((t1 - t0) * 1e3, (t2 - t1) * 1e3, fallback))
        score_ms = float(np.median([a for a, _, _ in times]))
        exact_ms = float(np.median([b for _, b, _ in times]))
        fb = times[-1][2]
        decisive = score_ms + exact_ms + sweep_ms / judge_every
        phase = decisive + (sweep_ms if fb else 0.0)
        pick = int(cand[int(np.argmax(np.abs(gc)))])
        out[tag] = {"score_rank_ms": round(score_ms, 3), "exact_ms": round(exact_ms, 3),
                    "n_exact": int(cand.size), "fallback": fb,
                    "judge_amortised_ms": round(sweep_ms / judge_every, 3),
                    "grad_phase_ms": round(phase, 3), "evals_per_s": round(n / (phase * 1e-3), 1),
                    "evals_per_s_without_fallback": round(n / (decisive * 1e-3), 1),
                    "pick_is_full_sweep_argmax": pick == kstar,
                    "argmax_rank": int(np.nonzero(order == kstar)[0][0])}
        del p, sg, fs
    out["plain_fp64_sweep_ms"] = round(sweep_ms, 3)
    out["plain_evals_per_s"] = round(n / (sweep_ms * 1e-3), 1)
    net.close()
    return out


def extras(hyp, torch, np, synth, S, H, ops, grad, w, M, na, nb):
    """Support skipping near Hartree-Fock and the device-side assembly."""
    bits = synth.near_hf_bits(M, na, nb, 24, seed=3)
    nidx = np.unique(S.rank(bits))
    rng_s = np.random.default_rng(11)
    nval = rng_s.standard_normal(nidx.size)
    nval /= np.sqrt(nval @ nval)
    psi_n = torch.zeros(S.dim, dtype=torch.float64, device="cuda")
    psi_n[torch.from_numpy(nidx).cuda()] = torch.from_numpy(nval).cuda()
    sig_n = torch.empty_like(psi_n)
    sup = {"state": f"Hartree-Fock + {nidx.size - 1} determinants one excitation away"}
    for on in (True, False):
        hyp.set_support_skip(on)
        hyp.hyp_apply_h(H, psi_n, sig_n)
        hyp.hyp_pool_gradients(S, ops, psi_n, sig_n, grad)
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        for _ in range(2):
            hyp.hyp_apply_h(H, psi_n, sig_n)
        torch.cuda.synchronize()
        t_b = time.perf_counter()
        for _ in range(2):
            hyp.hyp_pool_gradients(S, ops, psi_n, sig_n, grad)
        torch.cuda.synchronize()
        t_c = time.perf_counter()
        tag = "skip" if on else "dense"
        sup[f"hpsi_ms_{tag}"] = round((t_b - t_a) / 2 * 1e3, 3)
        sup[f"sweep_ms_{tag}"] = round((t_c - t_b) / 2 * 1e3, 3)
    hyp.set_support_skip(True)
    del psi_n, sig_n
    print(f"[bench] near Hartree-Fock: {sup}", file=sys.stderr, flush=True)

    # device-side Jordan-Wigner assembly of the workload's integrals
    _, _, _, h_int, g_int = synth.hamiltonian(w)
    hyp.hyp_assemble_pauli(h_int, g_int)
    torch.cuda.synchronize()
    t_a = time.perf_counter()
    n_asm = hyp.hyp_assemble_pauli(h_int, g_int)[0].size
    asm = {"terms": int(n_asm), "device_ms": round((time.perf_counter() - t_a) * 1e3, 2)}

    return sup, asm


def adapt_early(w, n_iter, skip_only=False):
    """Plain FP64 ADAPT iterations from Hartree-Fock (full sweep + BFGS),
    with support skipping on and then off: per-iteration wall time, its
    gradient and optimiser phases, the state's fill (nonzero amplitudes over
    the sector dimension), the cumulative time T_j and the paper's amortised
    iteration coefficient j / sqrt(T_j), and the selections (which must
    agree)."""
    import torch
    import synth
    import paper_2604_01176_amd as hyp

    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, _, _ = synth.hamiltonian(w)
    cre, ann, _ = synth.canonical_pool(M)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    probe = torch.from_numpy(synth.random_state(S.dim, 7)).cuda()
    H.tune(probe, reps=1)
    del probe
    runs = {}
    psi = torch.empty(S.dim, dtype=torch.float64, device="cuda")
    for on in ((True,) if skip_only else (True, False)):
        hyp.set_support_skip(on)
        A = hyp.Adapt(H, cre, ann, max_iter=n_iter + 1)
        rec = []
        t_cum = 0.0
        for it in range(n_iter):
            torch.cuda.synchronize()
            t1 = time.time()
            r = A.iterate()
            t2 = time.time()
            t_cum += t2 - t1
            rec.append(r)
            A.state(psi)
            fill = float((psi != 0).sum().item()) / S.dim
            print(json.dumps({"support_skip": on, "iteration": it, "selected": r["selected"], "E": r["energy"],
                              "grad_ms": round(r["grad_ms"], 1), "opt_ms": round(r["opt_ms"], 1),
                              "n_evals": r["n_evals"], "iter_s": round(t2 - t1, 3), "fill": fill,
                              "T_j_s": round(t_cum, 3), "j_over_sqrt_T": round((it + 1) / t_cum ** 0.5, 3)}),
                  flush=True)
            if r["selected"] < 0:
                break
        runs[on] = rec
    hyp.set_support_skip(True)
    if skip_only:
        return
    same = [a["selected"] == b["selected"] for a, b in zip(runs[True], runs[False])]
    print(json.dumps({"same_selections": same,
                      "dE_final": runs[True][-1]["energy"] - runs[False][-1]["energy"]}), flush=True)


def adapt_compare(w, n_iter, shadow=False):
    """The screen is trained on the GPU with the library's own kernels on
    exact sweeps of the 8-, 16- and 24-qubit workloads and the eight batch
    instances (floored residual targets, 16 epochs); then on the target
    workload: one plain FP64 ADAPT iteration per step (full sweep + BFGS)
    against screened FP32 iterations (top-512 + 256 audit, full sweep on the
    judge iterations, BFGS)."""
    import numpy as np
    import torch
    import synth
    import paper_2604_01176_amd as hyp
    from paper_2604_01176_amd import screen as scr

    t0 = time.time()
    Xs, ts = [], []
    train_set = [(synth.WORKLOADS[n], it) for n, it in (("h4_8q", 8), ("h8_16q", 8), ("h12_24q", 6))]
    train_set += [(v, 8) for v in synth.INSTANCES]
    for k, (v, iters) in enumerate(train_set):
        x, z, c, h, g = synth.hamiltonian(v)
        cre, ann, cls = synth.canonical_pool(v.n_orb)
        S = hyp.Sector(v.n_orb, v.n_alpha, v.n_beta)
        H = hyp.Hamiltonian(S, x, z, c)
        A = hyp.Adapt(H, cre, ann, max_iter=iters + 1)
        stat, qidx = scr.static_features(v.n_orb, cre, ann, cls, h, g)
        X, t = scr.collect_rows(A, scr.FeatureState(S, stat, qidx), iters, seed=k)
        Xs.append(X)
        ts.append(t)
    X = np.concatenate(Xs)
    t = np.concatenate(ts)
    net = scr.MLP(synth.mlp_init(0), 1 << 16)
    losses = scr.train(net, X, t, epochs=16, batch=1024, lr=1e-3)
    print(json.dumps({"screen_training_rows": int(X.shape[0]), "losses": [round(l, 4) for l in losses],
                      "train_s": round(time.time() - t0, 1)}), flush=True)

    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, h, g = synth.hamiltonian(w)
    cre, ann, cls = synth.canonical_pool(M)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    probe = torch.from_numpy(synth.random_state(S.dim, 7)).cuda()
    t64, _ = H.tune(probe, reps=1)
    t32, _ = H.tune(probe.float(), reps=1)
    del probe
    print(json.dumps({"hpsi_threads_fp64": t64, "hpsi_threads_fp32": t32}), flush=True)
    A64 = hyp.Adapt(H, cre, ann, max_iter=n_iter + 1)
    A32 = hyp.Adapt(H, cre, ann, dtype="f32", max_iter=n_iter + 1)
    stat, qidx = scr.static_features(M, cre, ann, cls, h, g)
    sc = scr.Screen(A32, S, stat, qidx, net, K=512, audit=256, judge_every=10, seed=42)
    for it in range(n_iter):
        torch.cuda.synchronize()
        t1 = time.time()
        r64 = A64.iterate()
        t2 = time.time()
        info = sc.iterate(it, shadow=shadow)
        t3 = time.time()
        print(json.dumps({"iteration": it, "plain_fp64": {"selected": r64["selected"], "E": r64["energy"],
                                                         "grad_ms": round(r64["grad_ms"], 1),
                                                         "opt_ms": round(r64["opt_ms"], 1),
                                                         "n_evals": r64["n_evals"],
                                                         "iter_s": round(t2 - t1, 2)},
                          "screened_fp32": {"selected": info["selected"], "E": info["energy"],
                                            "judge": info["judge"], "cheaper_full": info["cheaper_full"],
                                            "fallback": info["fallback"],
                                            "grad_phase_ms": round(info["grad_phase_ms"], 1),
                                            "n_exact": info["n_exact"], "grad_ms": round(info["grad_ms"], 1),
                                            "opt_ms": round(info["opt_ms"], 1), "n_evals": info["n_evals"],
                                            "iter_s": round(t3 - t2, 2),
                                            **({"shadow_agree": info.get("shadow_agree"),
                                                "shadow_in_candidates": info.get("shadow_in_candidates"),
                                                "shadow_rank": info.get("shadow_rank")} if shadow else {})},
                          "same_selection": r64["selected"] == info["selected"]}), flush=True)
    # FP64 polish of the screened run's ansatz
    ops, th = A32.ansatz()
    Ap = hyp.Adapt(H, cre, ann, max_iter=n_iter + 1)
    Ap.set_ansatz(ops, th)
    t4 = time.time()
    rp = Ap.optimize()
    print(json.dumps({"final_E_plain_fp64": A64.energy_fp64(), "final_E_screened_fp32_replayed_fp64": A32.energy_fp64(),
                      "dE": A32.energy_fp64() - A64.energy_fp64(), "final_E_screened_polished_fp64": rp["energy"],
                      "dE_polished": rp["energy"] - A64.energy_fp64(), "polish_s": round(time.time() - t4, 2),
                      "polish_evals": rp["n_evals"]}), flush=True)


def cpu_study(budget_s=20.0):
    """The CPU oracle (plain C + OpenMP, FP64, term by term / pair by pair)
    timed on this host at 1 thread and at all threads: H psi (every output
    row up to 24 qubits, a random row sample above, scaled), the pool sweep
    (every generator at 8 and 16 qubits, a random sample of generators above,
    scaled by the sample's share), and one ADAPT iteration (gradients +
    scipy BFGS) at 8 and 16 qubits.  Rates in the benchmark's units."""
    import numpy as np
    import synth
    import oracle
    from oracle.adapt import SectorProblem, run_adapt

    all_threads = oracle.max_threads()
    for name in ("h4_8q", "h8_16q", "h12_24q", "h14_28q", "h16_32q"):
        w = synth.WORKLOADS[name]
        M, na, nb = w.n_orb, w.n_alpha, w.n_beta
        x, z, c, _, _ = synth.hamiltonian(w)
        cre, ann, _ = synth.canonical_pool(M)
        m = model(M, na, nb, len(c), len(cre))
        dim = m["dim"]
        psi = synth.random_state(dim, 7)
        rng = np.random.default_rng(1)
        for th in (1, all_threads):
            oracle.set_threads(th)
            out = {"workload": name, "threads": th}
            # H psi: all rows if cheap, else a sample sized to about budget_s / 4
            rows = None if dim <= 5000 else rng.integers(0, dim, 2048)
            t0 = time.time()
            oracle.apply_h(M, na, nb, x, z, c, psi, out_idx=rows)
            dt = time.time() - t0
            frac = 1.0 if rows is None else rows.size / dim
            out["hpsi_s"] = round(dt / frac, 3)
            out["hpsi_gbs_gather_model"] = round(hpsi_gather_bytes(m) * frac / dt / 1e9, 4)
            # sweep: all generators if dim is small, else a sample
            if dim <= 5000:
                k = np.arange(len(cre))
            else:
                nk = 128 if dim <= 1_000_000 else (16 if dim <= 20_000_000 else 4)
                k = rng.choice(len(cre), size=min(len(cre), nk), replace=False)
            if True:
                # the sweep's cost does not depend on the values: psi stands in
                # for sigma above the small sizes
                sig = oracle.apply_h(M, na, nb, x, z, c, psi) if dim <= 5000 else psi
                t0 = time.time()
                oracle.pool_gradients(M, na, nb, cre[k], ann[k], psi, sig)
                dt = time.time() - t0
                out["sweep_s"] = round(dt * len(cre) / k.size, 2)
                out["sweep_evals_per_s"] = round(k.size / dt, 2)
                out["sweep_sampled_generators"] = int(k.size)
            if dim <= 5000:
                prob = SectorProblem(M, na, nb, x, z, c, cre, ann)
                t0 = time.time()
                run_adapt(prob, 1)
                out["adapt_first_iteration_s"] = round(time.time() - t0, 3)
            print(json.dumps(out), flush=True)
    oracle.set_threads(all_threads)


def graph_bench(reps=40):
    """One inner-optimiser evaluation E(theta), dE/dtheta (state preparation
    by j rotations, H psi, energy, adjoint gradient: 3j + O(1) launches)
    replayed from a captured hipGraph against the same launches issued
    eagerly; host wall time per evaluation over `reps` evaluations with
    fresh parameters (each evaluation waits for its energy and gradient)."""
    import numpy as np
    import torch
    import synth
    import paper_2604_01176_amd as hyp

    for name, js in (("h4_8q", (8, 32)), ("h8_16q", (8, 32)), ("h12_24q", (8, 32))):
        w = synth.WORKLOADS[name]
        x, z, c, _, _ = synth.hamiltonian(w)
        cre, ann, _ = synth.canonical_pool(w.n_orb)
        S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
        H = hyp.Hamiltonian(S, x, z, c)
        rng = np.random.default_rng(5)
        for j in js:
            ops = rng.choice(len(cre), size=j, replace=False).astype(np.int32)
            out = {"workload": name, "dim": S.dim, "parameters": j}
            for use_graph in (True, False):
                A = hyp.Adapt(H, cre, ann, max_iter=j + 1, use_graph=use_graph)
                A.set_ansatz(ops, rng.uniform(-0.3, 0.3, j))
                A.eval(rng.uniform(-0.3, 0.3, j))  # capture / warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    A.eval(rng.uniform(-0.3, 0.3, j))
                out["graph_ms" if use_graph else "eager_ms"] = round((time.perf_counter() - t0) / reps * 1e3, 3)
                A.close()
            out["speedup"] = round(out["eager_ms"] / out["graph_ms"], 2)
            print(json.dumps(out), flush=True)


def csr_bench(reps=5):
    """The paper's storage (the sector Hamiltonian materialised in CSR)
    against the matrix-free product on the same state: build time, SpMV and
    H psi times (HIP events), bytes; the 28-qubit CSR is refused for memory."""
    import torch
    import synth
    import paper_2604_01176_amd as hyp

    for name in ("h12_24q", "h14_28q"):
        w = synth.WORKLOADS[name]
        x, z, c, _, _ = synth.hamiltonian(w)
        S = hyp.Sector(w.n_orb, w.n_alpha, w.n_beta)
        H = hyp.Hamiltonian(S, x, z, c)
        psi = torch.from_numpy(synth.random_state(S.dim, 7)).cuda()
        out = {"workload": name, "dim": S.dim}
        try:
            t0 = time.perf_counter()
            A = hyp.CsrMatrix(H)
            out["build_s"] = round(time.perf_counter() - t0, 3)
        except hyp.HypError as e:
            out["csr"] = f"refused: {e}"
            print(json.dumps(out), flush=True)
            continue
        out["nnz"] = A.nnz
        out["csr_gb"] = round(A.nnz * 12 / 1e9, 2)
        y1, y2 = A.apply(psi), H.apply(psi)
        for tag, fn in (("csr_spmv_ms", lambda: A.apply(psi, y1)), ("matrix_free_ms", lambda: H.apply(psi, y2))):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            out[tag] = round(e0.elapsed_time(e1) / reps, 3)
        out["csr_stream_gbs"] = round(A.nnz * 12 / (out["csr_spmv_ms"] * 1e-3) / 1e9, 1)
        out["max_rel_diff"] = float((y1 - y2).norm() / y2.norm())
        print(json.dumps(out), flush=True)
        A.close()


def batch_bench(reps=5):
    """Eight uneven instances (M = 8..12), each with its full pool on a random
    state and its sigma: one persistent batched launch with the autotuned tile
    against the per-instance sweeps (the library's automatic strategy), both
    timed with HIP events on the library's stream; FP64."""
    import numpy as np
    import torch
    import synth
    import paper_2604_01176_amd as hyp

    jobs, total = [], 0
    for i, v in enumerate(synth.INSTANCES):
        x, z, c, _, _ = synth.hamiltonian(v)
        cre, ann, _ = synth.canonical_pool(v.n_orb)
        S = hyp.Sector(v.n_orb, v.n_alpha, v.n_beta)
        H = hyp.Hamiltonian(S, x, z, c)
        psi = torch.from_numpy(synth.random_state(S.dim, 100 + i)).cuda()
        sig = H.apply(psi)
        ops = hyp.exc_tensor(cre, ann)
        g = torch.empty(len(cre), dtype=torch.float64, device="cuda")
        jobs.append((S, ops, psi, sig, g, H))
        total += len(cre)
    bj = [j[:5] for j in jobs]
    tile, tune_ms = hyp.hyp_tune_pool_gradients(bj, reps=2)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_batched = timed(lambda: hyp.hyp_pool_gradients_batched(bj, tile))
    g_batched = [j[4].clone() for j in jobs]

    def per_instance():
        for S, ops, psi, sig, g, _ in jobs:
            hyp.hyp_pool_gradients(S, ops, psi, sig, g)
    ms_single = timed(per_instance)
    dev = max(float((a - j[4]).abs().max()) / max(1.0, float(j[4].abs().max())) for a, j in zip(g_batched, jobs))
    try:
        hyp.set_sweep_mode("pairs")
        ms_fused_full = timed(lambda: hyp.hyp_pool_gradients_batched(bj, tile))
    finally:
        hyp.set_sweep_mode("auto")
    # candidate subsets (768 per instance, the screen's K + audit): fused launch vs per-instance calls
    rng = np.random.default_rng(5)
    sub = []
    for S, ops, psi, sig, g, _ in jobs:
        k = torch.from_numpy(np.sort(rng.choice(ops.shape[0], min(768, ops.shape[0] // 5), replace=False))).cuda()
        sub.append((S, ops.index_select(0, k).contiguous(), psi, sig,
                    torch.empty(k.shape[0], dtype=torch.float64, device="cuda")))
    n_sub = sum(j[1].shape[0] for j in sub)
    tile_sub, _ = hyp.hyp_tune_pool_gradients(sub, reps=2)
    ms_sub_fused = timed(lambda: hyp.hyp_pool_gradients_batched(sub, tile_sub))

    def sub_single():
        for S, ops, psi, sig, g in sub:
            hyp.hyp_pool_gradients(S, ops, psi, sig, g)
    ms_sub_single = timed(sub_single)
    print(json.dumps({"instances": [f"M={v.n_orb} ({v.n_alpha},{v.n_beta})" for v in synth.INSTANCES],
                      "full_pools": {"generators": total, "batched_ms": round(ms_batched, 3),
                                     "batched_evals_per_s": round(total / (ms_batched * 1e-3), 1),
                                     "per_instance_ms": round(ms_single, 3),
                                     "fused_pair_launch_ms": round(ms_fused_full, 3), "tile": list(tile),
                                     "max_rel_diff": dev},
                      "candidate_subsets": {"generators": n_sub, "fused_ms": round(ms_sub_fused, 3),
                                            "fused_evals_per_s": round(n_sub / (ms_sub_fused * 1e-3), 1),
                                            "per_instance_ms": round(ms_sub_single, 3), "tile": list(tile_sub)}}),
          flush=True)


def fp32_study(w, n_iter):
    """FP64 ADAPT run; at every iteration the FP32-storage path is evaluated on
    the same ansatz and parameters: H psi relative error, energy error,
    pool-gradient error; then an independent FP32 run's final energy."""
    import numpy as np
    import torch
    import synth
    import paper_2604_01176_amd as hyp

    M, na, nb = w.n_orb, w.n_alpha, w.n_beta
    x, z, c, _, _ = synth.hamiltonian(w)
    cre, ann, _ = synth.canonical_pool(M)
    S = hyp.Sector(M, na, nb)
    H = hyp.Hamiltonian(S, x, z, c)
    A64 = hyp.Adapt(H, cre, ann, max_iter=n_iter + 1)
    A32 = hyp.Adapt(H, cre, ann, dtype="f32", max_iter=n_iter + 1)
    p64 = p32 = None
    for it in range(n_iter):
        t = time.time()
        r = A64.gradients(None)
        g64 = A64.last_gradients()
        ops, th = A64.ansatz()
        A32.set_ansatz(ops, th)
        r32 = A32.gradients(None)
        g32 = A32.last_gradients()
        p64 = A64.state(p64)
        p32 = A32.state(p32)
        s64 = H.apply(p64)
        s32 = H.apply(p32)
        hpsi_err = float(torch.linalg.norm(s32.double() - s64) / torch.linalg.norm(s64))
        e_err = r32["energy_before"] - r["energy_before"]
        rec = A64.select_optimize()
        print(json.dumps({"iteration": it, "E64": r["energy_before"], "dE_fp32": e_err,
                          "hpsi_rel_err": hpsi_err, "max_dg": float(np.max(np.abs(g32 - g64))),
                          "gmax": r["gmax"], "argmax_same": int(np.argmax(np.abs(g32)) == np.argmax(np.abs(g64))),
                          "selected": rec["selected"], "wall_s": round(time.time() - t, 2)}), flush=True)
        if rec["selected"] < 0:
            break
    B32 = hyp.Adapt(H, cre, ann, dtype="f32", max_iter=n_iter + 1)
    for it in range(n_iter):
        if B32.iterate()["selected"] < 0:
            break
    print(json.dumps({"final_E64": A64.energy_fp64(), "final_E_fp32_run_replayed_fp64": B32.energy_fp64(),
                      "dE_final": B32.energy_fp64() - A64.energy_fp64(),
                      "same_selections": bool(np.array_equal(A64.ansatz()[0], B32.ansatz()[0]))}), flush=True)


if __name__ == "__main__":
    main()
