"""Benchmark: Laplace FMM on one MI355X.

One step = build the octree + evaluate potentials and fields (every step of
the forward path: keys, level selection, sort, P2M, M2M, M2L, L2L, L2P, P2P,
combine) for N = 1e6 particles uniform in the unit cube, charges U[0,1),
p = 10, leaf <= 64, inputs resident in HBM.  Prints one JSON line.

  value        particles/s of the mixed form (N / step time)
  p2p_gint_s   P2P Ginteractions/s (mixed), pairs from the tree / P2P time
  fp64         the plain FP64 form measured the same way
  rel_l2       errors vs the FP64 direct sum on 1000 sampled targets
  roofline     dominant kernel of the mixed step (M2L or P2P, whichever
               stage is longer in stages_ms); its duration is the mean of
               HIP events that the library records around that stage only
               (each event marker idles the GPU for a few microseconds) on
               the stream its kernels run on, during the timed steps
  stages_ms    all stages, from a separate fully profiled run before the
               timed steps
  roofline_p2p the same for the other kernel (roofline_m2l when P2P
               dominates), its duration from stages_ms; traffic only on the
               workload the counter summaries were taken on
  cpu_baseline the CPU oracle FMM on the host cores
  adjoint      forward + backward throughput of the differentiable form
               (N = 1e6, p = 8, leaf <= 64)
  small        the small case (N = 1e4, p = 4, leaf <= 64), where launch
               latency dominates: evaluate and build + evaluate, eager, with
               a replayed HIP graph, and with the concurrent near field

--copy-probe runs a device-to-device copy of a known size (for scaling the
FETCH_SIZE / WRITE_SIZE counters of rocprofv3 to bytes).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2 (dual issue) x 2.4 GHz
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
P2P_FLOP_PER_PAIR = 19
COPY_PROBE_BYTES = 1 << 30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="particles for the CPU oracle baseline (0: the whole workload)")
    ap.add_argument("--splits", type=int, default=3, help="bf16 parts of the mixed M2L (2 or 3)")
    ap.add_argument("--copy-probe", action="store_true")
    return ap.parse_args()


def timed_steps(step, steps, warmup, sync):
    for _ in range(warmup):
        step()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    sync()
    return (time.perf_counter() - t0) / steps


def traffic_from_profile(kernel_file, summary):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None when it is missing or was taken on another version of the kernel."""
    path = os.path.join(ROOT, "profiles", summary)
    src = os.path.join(ROOT, "paper_1106_2176_amd", "csrc", kernel_file)
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("source_sha256") != sha:
        return None
    try:
        fetch = float(kv["fetch_kib_per_dispatch"]) / float(kv["copy_fetch_factor"])
        write = float(kv["write_kib_per_dispatch"]) / float(kv["copy_write_factor"])
    except (KeyError, ValueError, ZeroDivisionError):
        return None
    return (fetch + write) * 1024.0


def copy_probe():
    import torch
    x = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": COPY_PROBE_BYTES, "copies": 3}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    import torch

    import paper_1106_2176_amd as fmm
    from paper_1106_2176_amd import inputs

    wl = inputs.WORKLOADS[args.workload]
    pos_np, q_np = inputs.workload(args.workload)
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_np).to(dev)
    q = torch.from_numpy(q_np).to(dev)
    sync = torch.cuda.synchronize

    def run_form(precision, steps, warmup):
        phi = torch.empty_like(q)
        E = torch.empty_like(pos)

        def timed(stages, nsteps, nwarm):
            tree = fmm.Tree(pos, p=wl.p, leaf_max=wl.leaf_max, precision=precision, profile=True,
                            profile_stages=stages, bf16_splits=args.splits)

            def step():
                tree.rebuild(pos)
                tree.evaluate(q, vec="field", phi=phi, out_vec=E)

            for _ in range(nwarm):
                step()
            tree.stage_times_reset()
            # stage times: library events over the timed steps (mean of the
            # last min(steps, 32) of them)
            sec = timed_steps(step, nsteps, 0, sync)
            st = tree.stage_times()
            info = tree.info()
            tree.close()
            return sec, st, info

        # every stage, outside the timed region; it names the dominant stage
        stages_ms = timed(None, max(5, steps // 2), max(1, warmup))[1]
        dom = "M2L" if stages_ms["M2L"] >= stages_ms["P2P"] else "P2P"
        # the timed steps: events only around the dominant (roofline) stage
        sec, roof_st, info = timed((dom,), steps, warmup)
        return {"sec": sec, "dom": dom, "dom_ms": roof_st[dom], "stages_ms": stages_ms, "info": info,
                "phi": phi.clone(), "E": E.clone()}

    mixed = run_form("mixed", args.steps, args.warmup)
    info = mixed["info"]
    n = wl.n
    value = n / mixed["sec"]
    # the dominant stage's time from the events of the timed steps, the
    # other's from the profiled run
    dom = mixed["dom"]
    p2p_ms = mixed["dom_ms"] if dom == "P2P" else mixed["stages_ms"]["P2P"]
    m2l_ms = mixed["dom_ms"] if dom == "M2L" else mixed["stages_ms"]["M2L"]
    # the counter summaries were taken on the default workload only
    on_profiled = args.workload == "C2" and args.splits == 3
    pairs = info["p2p_pairs"]
    m2l_pairs = info["m2l_pairs"]
    p2p_tflops = P2P_FLOP_PER_PAIR * pairs / (p2p_ms * 1e-3) / 1e12
    m2l_tflops = 2.0 * wl.p ** 4 * m2l_pairs / (m2l_ms * 1e-3) / 1e12
    roof_p2p = {"kernel": "k_p2p<float>", "bound": "alu", "achieved": p2p_tflops,
                "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": p2p_tflops / PEAK_FP32_VECTOR_TFLOPS,
                "traffic": traffic_from_profile("p2p.hip", "p2p_C2_traffic.txt") if on_profiled else None,
                "ms": p2p_ms, "flop_per_launch": P2P_FLOP_PER_PAIR * pairs}
    split_products = {3: 6, 2: 3}.get(args.splits, 6)
    roof_m2l = {"kernel": "k_m2l_bf16<%d,%d>" % (args.splits, wl.p), "bound": "mfma",
                "achieved": m2l_tflops, "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": m2l_tflops / PEAK_BF16_MFMA_TFLOPS,
                "traffic": traffic_from_profile("m2l.hip", "m2l_bf16_C2_traffic.txt") if on_profiled else None,
                "ms": m2l_ms, "flop_per_launch": 2.0 * wl.p ** 4 * m2l_pairs,
                "bf16_products_per_term": split_products}
    roof = roof_m2l if dom == "M2L" else roof_p2p

    # accuracy on sampled targets vs the FP64 direct sum
    t_idx = inputs.targets(n, wl.seed)
    import oracle
    phi_d, E_d = oracle.direct(pos_np, q_np, t_idx)

    def errs(res):
        ph = res["phi"].cpu().numpy()[t_idx]
        Ef = res["E"].cpu().numpy()[t_idx]
        qq = q_np[t_idx][:, None]
        return {"phi": float(np.linalg.norm(ph - phi_d) / np.linalg.norm(phi_d)),
                "F": float(np.linalg.norm(qq * (Ef - E_d)) / np.linalg.norm(qq * E_d))}

    rel = {"mixed_vs_direct": errs(mixed)}
    fp64 = None
    if not args.no_fp64:
        fp64 = run_form("fp64", max(3, args.steps // 4), 1)
        rel["fp64_vs_direct"] = errs(fp64)
        a, b = mixed["phi"].cpu().numpy(), fp64["phi"].cpu().numpy()
        Ea, Eb = mixed["E"].cpu().numpy(), fp64["E"].cpu().numpy()
        qq = q_np[:, None]
        rel["mixed_vs_fp64_all"] = {
            "phi": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
            "F": float(np.linalg.norm(qq * (Ea - Eb)) / np.linalg.norm(qq * Eb))}

    adj = None
    if not args.no_adjoint:
        w5 = inputs.WORKLOADS["C5"]
        p5, q5 = inputs.workload("C5")
        wv = torch.from_numpy(inputs.weights(w5.n, w5.seed)).to(dev)
        P5 = torch.from_numpy(p5).to(dev)
        Q5 = torch.from_numpy(q5).to(dev)
        tree5 = fmm.Tree(P5, p=w5.p, leaf_max=w5.leaf_max, precision="mixed")

        def fb():
            tree5.rebuild(P5)
            _, E5 = tree5.evaluate(Q5)
            tree5.rebuild(P5)  # the tree is recomputed for the backward pass
            tree5.backward(Q5, wv, E5)

        s5 = timed_steps(fb, max(3, args.steps // 2), 2, sync)
        tree5.close()
        adj = {"workload": w5.describe() + ", loss sum w_i phi_i, w ~ N(0,1)",
               "fwd_bwd_particles_per_s": w5.n / s5, "ms_per_step": s5 * 1e3}

    small = None
    if not args.no_small:
        w1 = inputs.WORKLOADS["C1"]
        p1, q1 = inputs.workload("C1")
        P1, Q1 = torch.from_numpy(p1).to(dev), torch.from_numpy(q1).to(dev)
        phi1 = torch.empty_like(Q1)
        E1 = torch.empty_like(P1)
        small = {"workload": w1.describe()}
        for name, kw in (("eager", {}), ("graph", {"graph": True}),
                         ("graph_overlap", {"graph": True, "overlap_near": True})):
            t1 = fmm.Tree(P1, p=w1.p, leaf_max=w1.leaf_max, precision="mixed", **kw)

            def ev():
                t1.evaluate(Q1, vec="field", phi=phi1, out_vec=E1)

            def st():
                t1.rebuild(P1)
                ev()

            small[name] = {"evaluate_us": 1e6 * timed_steps(ev, 200, 10, sync),
                           "step_us": 1e6 * timed_steps(st, 100, 5, sync)}
            t1.close()

    cpu = None
    if not args.no_cpu:
        ns = args.cpu_sample if args.cpu_sample > 0 else n
        ps, qs = inputs.particles(ns, wl.seed, wl.charges, wl.dtype)
        t0 = time.perf_counter()
        oracle.fmm(ps.astype(np.float64), qs.astype(np.float64), wl.p, wl.leaf_max)
        tc = time.perf_counter() - t0
        what = "the whole workload" if ns == n else "a sample of N=%d particles" % ns
        cpu = {"value": ns / tc, "unit": "particles/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "FP64 Cartesian-Taylor oracle FMM (OpenMP) on %s of the same "
                         "distribution, p=%d, leaf<=%d: %.1f s" % (what, wl.p, wl.leaf_max, tc)}

    line = {
        "metric": "particles/s + P2P Ginteractions/s at 1e-6 rel-L2, mixed vs FP64 on 1 GPU",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["sec"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16(split)+f64",
        "data": "synthetic",
        "config": {"workload": wl.describe(), "form": "mixed", "bf16_splits": args.splits,
                   "levels": info["levels"],
                   "p2p_pairs": pairs, "m2l_pairs": m2l_pairs},
        "p2p_gint_s": pairs / (p2p_ms * 1e-3) / 1e9,
        "stages_ms": mixed["stages_ms"],
        "roofline": roof,
        ("roofline_p2p" if dom == "M2L" else "roofline_m2l"): roof_p2p if dom == "M2L" else roof_m2l,
        "rel_l2": rel,
        "cpu_baseline": cpu,
        "adjoint": adj,
        "small": small,
    }
    if fp64 is not None:
        line["fp64"] = {"particles_per_s": n / fp64["sec"], "ms_per_step": fp64["sec"] * 1e3,
                        "p2p_gint_s": pairs / (fp64["stages_ms"]["P2P"] * 1e-3) / 1e9,
                        "stages_ms": fp64["stages_ms"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
