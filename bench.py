"""Benchmark: Laplace FMM on one MI355X.

One step = build the octree + evaluate potentials and fields (every step of
the forward path: keys, level selection, sort, P2M, M2M, M2L, L2L, L2P, P2P,
combine) for N = 1e6 particles uniform in the unit cube, charges U[0,1),
p = 10, leaf <= 64, inputs resident in HBM.  Prints one JSON line.

  value        particles/s of the mixed form (N / step time)
  p2p_gint_s   P2P Ginteractions/s (mixed), pairs from the tree / P2P time
  fp64         the plain FP64 form measured the same way
  rel_l2       errors vs the FP64 direct sum on 1000 sampled targets, and
               mixed vs FP64 on all N
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
  tree_pass    the HBM-bound passes (build, P2M with the charge gather, L2P,
               combine): algorithmic bytes over their time; tree_pass_c4_counters
               the same kernels at N = 1e8 with measured HBM bytes from the
               committed rocprofv3 counter summary
  overlap      the same step with the near field on a concurrent stream
  c3           N = 1e7, p = 10, leaf <= 128, zero-mean charges: both forms,
               their dominant kernel, errors vs the direct sum and each other
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

# 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s issuing one
# FP32 instruction per lane and cycle; the published 157.3 counts packed
# (two-wide) FP32, which this build does not use
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_16BIT_MFMA_TFLOPS = 2500.0  # bf16 and fp16 dense
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
P2P_FLOP_PER_PAIR = 19
# stage names of fmm_stage_times, and their meaning on an adaptive tree
STAGE_NAMES = ("gather", "P2M", "M2M", "pack", "M2L", "L2L", "L2P", "P2P", "combine")
ADAPTIVE_STAGE_NAMES = ("gather", "P2M", "M2M", "P2L", "M2L", "L2L", "L2P+M2P", "P2P", "combine")
COPY_PROBE_BYTES = 1 << 30

# mixed-form M2L encodings: tree options and MFMA products per term
ENCODINGS = {"fp16x2": ({"m2l_fp16": True}, 3),
             "bf16x3": ({"m2l_fp16": False, "bf16_splits": 3}, 6),
             "bf16x2": ({"m2l_fp16": False, "bf16_splits": 2}, 3)}


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
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-overlap", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="particles for the CPU oracle baseline (0: the whole workload)")
    ap.add_argument("--m2l", default="fp16x2", choices=sorted(ENCODINGS),
                    help="M2L operand encoding of the mixed form")
    ap.add_argument("--copy-probe", action="store_true")
    return ap.parse_args()


def log(msg):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def timed_steps(step, steps, warmup, sync):
    for _ in range(warmup):
        step()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    sync()
    return (time.perf_counter() - t0) / steps


def read_profile(summary, kernel_file):
    """key: value pairs of a committed rocprofv3 summary, or None when it is
    missing or was taken on another version of the kernel's source."""
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
    return kv if kv.get("source_sha256") == sha else None


def traffic_from_profile(kernel_file, summary):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, each divided by its
    copy-kernel factor) from a committed counter summary, or None."""
    kv = read_profile(summary, kernel_file)
    if kv is None:
        return None
    try:
        fetch = float(kv["fetch_kib_per_dispatch"]) / float(kv["copy_fetch_factor"])
        write = float(kv["write_kib_per_dispatch"]) / float(kv["copy_write_factor"])
    except (KeyError, ValueError, ZeroDivisionError):
        return None
    return (fetch + write) * 1024.0


def tree_pass_counters():
    """The tree passes at N = 1e8 (C4) from the committed counter summary:
    per kernel the mean duration, measured HBM bytes (FETCH_SIZE + WRITE_SIZE,
    scaled) and algorithmic bytes, or None when the summary is missing or the
    kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "tree_passes_C4_traffic.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    csrc = os.path.join(ROOT, "paper_1106_2176_amd", "csrc")
    for name in ("tree.hip", "far.hip"):
        sha = hashlib.sha256(open(os.path.join(csrc, name), "rb").read()).hexdigest()
        if "%s %s" % (name, sha) not in text:
            return None
    out = {}
    for line in text.splitlines():
        f = line.replace("(", " ").replace(")", " ").replace("+", " ").split()
        if line.startswith("#") or len(f) < 6:
            continue
        if f[0] == "total":
            out["total"] = {"us": float(f[1]), "measured_mb": float(f[2]), "algorithmic_mb": float(f[3]),
                            "measured_gbs": float(f[4]), "algorithmic_gbs": float(f[5])}
        else:
            out[f[0]] = {"us": float(f[1]), "measured_mb": float(f[2]), "algorithmic_mb": float(f[5]),
                         "measured_gbs": float(f[6]), "algorithmic_gbs": float(f[7])}
    return out or None


def copy_probe():
    import torch
    x = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": COPY_PROBE_BYTES, "copies": 3}), flush=True)


def measure(fmm, wl, pos, q, precision, steps, warmup, sync, **kw):
    """Build + evaluate steps of one form: every stage's time from a fully
    profiled run (outside the timed region), then the timed steps with events
    only around the dominant stage (M2L or P2P)."""
    import torch
    phi = torch.empty_like(q)
    E = torch.empty_like(pos)

    def run(stages, nsteps, nwarm):
        tree = fmm.Tree(pos, p=wl.p, leaf_max=wl.leaf_max, precision=precision, profile=True,
                        profile_stages=stages, **kw)

        def step():
            tree.rebuild(pos)
            tree.evaluate(q, vec="field", phi=phi, out_vec=E)

        for _ in range(nwarm):
            step()
        tree.stage_times_reset()
        sec = timed_steps(step, nsteps, 0, sync)
        st = tree.stage_times()
        info = tree.info()

        def build():
            tree.rebuild(pos)
        build_s = timed_steps(build, max(3, nsteps // 2), 1, sync)
        tree.close()
        return sec, st, info, build_s

    stages_ms = run(None, max(5, steps // 2), max(1, warmup))[1]
    dom = "M2L" if stages_ms["M2L"] >= stages_ms["P2P"] else "P2P"
    sec, roof_st, info, build_s = run((dom,), steps, warmup)
    return {"sec": sec, "dom": dom, "dom_ms": roof_st[dom], "stages_ms": stages_ms, "info": info,
            "build_ms": build_s * 1e3, "phi": phi.clone(), "E": E.clone()}


def rooflines(wl, res, precision, enc, on_profiled):
    """(dominant-kernel roofline, the other one) of a measured form."""
    info, dom = res["info"], res["dom"]
    p2p_ms = res["dom_ms"] if dom == "P2P" else res["stages_ms"]["P2P"]
    m2l_ms = res["dom_ms"] if dom == "M2L" else res["stages_ms"]["M2L"]
    pairs, m2l_pairs = info["p2p_pairs"], info["m2l_pairs"]
    p2p_tf = P2P_FLOP_PER_PAIR * pairs / (p2p_ms * 1e-3) / 1e12
    m2l_tf = 2.0 * wl.p ** 4 * m2l_pairs / (m2l_ms * 1e-3) / 1e12
    f64 = precision == "fp64"
    p2p = {"kernel": "k_p2p<%s>" % ("double" if f64 else "float"), "bound": "alu", "achieved": p2p_tf,
           "peak": PEAK_FP64_TFLOPS if f64 else PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
           "frac": p2p_tf / (PEAK_FP64_TFLOPS if f64 else PEAK_FP32_VECTOR_TFLOPS),
           "traffic": traffic_from_profile("p2p.hip", "p2p_C2_counters.txt") if on_profiled and not f64 else None,
           "ms": p2p_ms, "flop_per_launch": P2P_FLOP_PER_PAIR * pairs}
    if not f64:
        p2p["peak_unpacked"] = PEAK_FP32_UNPACKED_TFLOPS
        p2p["frac_unpacked"] = p2p_tf / PEAK_FP32_UNPACKED_TFLOPS
    if f64:
        m2l = {"kernel": "k_m2l_f64<%d>" % wl.p, "bound": "mfma", "achieved": m2l_tf,
               "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": m2l_tf / PEAK_FP64_TFLOPS,
               "traffic": None}
    else:
        opts, products = ENCODINGS[enc]
        nparts = 2 if opts.get("m2l_fp16") else opts["bf16_splits"]
        m2l = {"kernel": "k_m2l_bf16<%d,%d,8,%s>" % (nparts, wl.p, "fp16" if opts.get("m2l_fp16") else "bf16"),
               "bound": "mfma", "achieved": m2l_tf, "peak": PEAK_16BIT_MFMA_TFLOPS, "unit": "TFLOP/s",
               "frac": m2l_tf / PEAK_16BIT_MFMA_TFLOPS,
               "traffic": traffic_from_profile("m2l.hip", "m2l_%s_C2_counters.txt" % enc) if on_profiled else None,
               "encoding": enc, "mfma_products_per_term": products}
    m2l.update({"ms": m2l_ms, "flop_per_launch": 2.0 * wl.p ** 4 * m2l_pairs})
    return (m2l, p2p) if dom == "M2L" else (p2p, m2l)


# The adaptive-tree record: Gaussian blobs (inputs.clustered), FP64 form,
# beside the uniform FP64 tree on the same input with its level capped at 7
# and at 8 (uncapped, the uniform level of these blobs would exceed 8).
ADAPTIVE = {"n": 1_000_000, "seed": 6, "blobs": 6, "p": 8, "leaf_max": 64, "max_level": 8,
            "uniform_levels": (7, 8)}


def sampled_errors(res, q_np, t_idx, phi_d, E_d):
    """Relative L2 of phi and F = qE on sampled targets against the direct sum."""
    ph = res["phi"].cpu().numpy().astype(np.float64)[t_idx]
    Ef = res["E"].cpu().numpy().astype(np.float64)[t_idx]
    qq = q_np.astype(np.float64)[t_idx][:, None]
    return {"phi": float(np.linalg.norm(ph - phi_d) / np.linalg.norm(phi_d)),
            "F": float(np.linalg.norm(qq * (Ef - E_d)) / np.linalg.norm(qq * E_d))}


def adaptive_rooflines(p, res):
    """(dominant, other) rooflines of the adaptive tree's M2L (gathered FP64
    MFMA, 2 p^4 FLOP per V entry) and P2P (FP64, 19 FLOP per pair)."""
    info, st = res["info"], res["stages_ms"]
    m2l_ms = res["dom_ms"] if res["dom"] == "M2L" else st["M2L"]
    p2p_ms = res["dom_ms"] if res["dom"] == "P2P" else st["P2P"]
    m2l_tf = 2.0 * p ** 4 * info["m2l_pairs"] / (m2l_ms * 1e-3) / 1e12
    p2p_tf = P2P_FLOP_PER_PAIR * info["p2p_pairs"] / (p2p_ms * 1e-3) / 1e12
    m2l = {"kernel": "k_ad_m2l<%d>" % p, "bound": "mfma", "achieved": m2l_tf, "peak": PEAK_FP64_TFLOPS,
           "unit": "TFLOP/s", "frac": m2l_tf / PEAK_FP64_TFLOPS, "traffic": None, "ms": m2l_ms,
           "flop_per_launch": 2.0 * p ** 4 * info["m2l_pairs"]}
    p2p = {"kernel": "k_ad_p2p", "bound": "alu", "achieved": p2p_tf, "peak": PEAK_FP64_TFLOPS,
           "unit": "TFLOP/s", "frac": p2p_tf / PEAK_FP64_TFLOPS, "traffic": None, "ms": p2p_ms,
           "flop_per_launch": P2P_FLOP_PER_PAIR * info["p2p_pairs"]}
    return (m2l, p2p) if res["dom"] == "M2L" else (p2p, m2l)


def adaptive_record(fmm, oracle, inputs, steps, warmup, sync, dev, overlap=True):
    import torch
    a = ADAPTIVE
    n = a["n"]
    pos_np, q_np = inputs.clustered(n, a["seed"], a["blobs"])
    P, Q = torch.from_numpy(pos_np).to(dev), torch.from_numpy(q_np).to(dev)
    wl = inputs.Workload("clustered", a["seed"], n, a["p"], a["leaf_max"], "u01", "f64")
    t_idx = inputs.targets(n, a["seed"])
    phi_d, E_d = oracle.direct(pos_np, q_np, t_idx)
    res = measure(fmm, wl, P, Q, "fp64", steps, warmup, sync, adaptive=True, max_level=a["max_level"])
    log("adaptive tree: adaptive form measured")
    info = res["info"]
    roof, other = adaptive_rooflines(a["p"], res)
    names = dict(zip(STAGE_NAMES, ADAPTIVE_STAGE_NAMES))
    out = {"workload": "N=%g Gaussian blobs (%d blobs, widths U[0.005,0.06)), charges U[0,1), p=%d, "
                       "leaf<=%d, max level %d, f64 positions/charges, FP64 form"
                       % (n, a["blobs"], a["p"], a["leaf_max"], a["max_level"]),
           "ms_per_step": res["sec"] * 1e3, "particles_per_s": n / res["sec"],
           "build_ms": res["build_ms"],
           "stages_ms": {names[k]: v for k, v in res["stages_ms"].items()},
           "tree": {k: info[k] for k in ("levels", "n_boxes", "n_leaves", "max_leaf_count", "p2p_pairs",
                                         "m2l_pairs", "m2p_evals", "p2l_evals")},
           "p2p_gint_s": info["p2p_pairs"] / (res["stages_ms"]["P2P"] * 1e-3) / 1e9,
           "roofline": roof, ("roofline_p2p" if res["dom"] == "M2L" else "roofline_m2l"): other,
           "rel_l2_vs_direct": sampled_errors(res, q_np, t_idx, phi_d, E_d), "uniform": {}}
    # the mixed form: the M2L in two binary16 parts (3 MFMA products), the rest FP64
    mix = measure(fmm, wl, P, Q, "mixed", steps, warmup, sync, adaptive=True, max_level=a["max_level"])
    log("adaptive tree: mixed form measured")
    ov = None
    if overlap:
        ov = measure(fmm, wl, P, Q, "mixed", steps, warmup, sync, adaptive=True, max_level=a["max_level"],
                     overlap_near=True)
        log("adaptive tree: mixed form with the concurrent near field measured")
    m2l_ms = mix["dom_ms"] if mix["dom"] == "M2L" else mix["stages_ms"]["M2L"]
    m2l_tf = 2.0 * a["p"] ** 4 * info["m2l_pairs"] / (m2l_ms * 1e-3) / 1e12
    out["mixed"] = {
        "ms_per_step": mix["sec"] * 1e3, "particles_per_s": n / mix["sec"], "build_ms": mix["build_ms"],
        "stages_ms": {names[k]: v for k, v in mix["stages_ms"].items()},
        "roofline_m2l": {"kernel": "k_ad_m2l_h<%d>" % a["p"], "bound": "mfma", "achieved": m2l_tf,
                         "peak": PEAK_16BIT_MFMA_TFLOPS, "unit": "TFLOP/s", "frac": m2l_tf / PEAK_16BIT_MFMA_TFLOPS,
                         "traffic": None, "ms": m2l_ms, "mfma_products_per_term": 3},
        "overlap_ms_per_step": ov["sec"] * 1e3 if ov else None,
        "rel_l2_vs_direct": sampled_errors(mix, q_np, t_idx, phi_d, E_d),
        "rel_l2_vs_fp64_all": {
            "phi": float(np.linalg.norm((mix["phi"] - res["phi"]).cpu().numpy()) /
                         np.linalg.norm(res["phi"].cpu().numpy())),
            "E": float(np.linalg.norm((mix["E"] - res["E"]).cpu().numpy()) / np.linalg.norm(res["E"].cpu().numpy()))}}
    del res, mix, ov
    for ml in a["uniform_levels"]:
        u = measure(fmm, wl, P, Q, "fp64", 2, 1, sync, max_level=ml)
        log("adaptive tree: uniform tree at max level %d measured" % ml)
        out["uniform"]["max_level_%d" % ml] = {
            "levels": u["info"]["levels"], "ms_per_step": u["sec"] * 1e3, "particles_per_s": n / u["sec"],
            "p2p_pairs": u["info"]["p2p_pairs"], "m2l_pairs": u["info"]["m2l_pairs"],
            "stages_ms": u["stages_ms"], "rel_l2_vs_direct": sampled_errors(u, q_np, t_idx, phi_d, E_d)}
        del u
    return out


def tree_pass(wl, res, precision):
    """Algorithmic HBM bytes of the build, P2M (with the charge gather) and
    L2P over their measured time (build: wall time of the rebuild, which
    includes its one host wait).  The combine is not among them: in the
    serial chain timed here the P2P kernel ends with it."""
    info = res["info"]
    n, nleaf = info["n"], info["n_leaves"]
    S = (wl.p * wl.p + 7) // 8 * 8
    inb = 12 if wl.dtype == "f32" else 24        # caller positions per particle
    qb = 4 if wl.dtype == "f32" else 8           # caller charge / potential
    rec = 32 if precision == "fp64" else 16      # sorted record
    cb = 8 if precision == "fp64" else 4         # leaf-level coefficient
    build = n * (inb + 8 + 12 + 4 + inb + 4 + rec)   # keys; place; fix-up
    p2m = n * (rec + 4 + qb + 4) + nleaf * S * cb    # records, perm, charges -> M_L
    l2p = n * (rec + 32) + nleaf * S * cb            # records, L_L -> far partials
    st = res["stages_ms"]
    ms = res["build_ms"] + st["gather"] + st["P2M"] + st["L2P"]
    total = build + p2m + l2p
    return {"bytes": total, "ms": ms, "gbs": total / (ms * 1e-3) / 1e9,
            "frac_hbm": total / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "build_ms": res["build_ms"]}


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

    import oracle
    import paper_1106_2176_amd as fmm
    from paper_1106_2176_amd import inputs

    wl = inputs.WORKLOADS[args.workload]
    pos_np, q_np = inputs.workload(args.workload)
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_np).to(dev)
    q = torch.from_numpy(q_np).to(dev)
    sync = torch.cuda.synchronize
    enc_kw = ENCODINGS[args.m2l][0]

    mixed = measure(fmm, wl, pos, q, "mixed", args.steps, args.warmup, sync, **enc_kw)
    log("%s mixed form measured" % args.workload)
    info = mixed["info"]
    n = wl.n
    value = n / mixed["sec"]
    # the counter summaries were taken on the default workload only
    on_profiled = args.workload == "C2"
    roof, other = rooflines(wl, mixed, "mixed", args.m2l, on_profiled)
    pairs = info["p2p_pairs"]
    p2p_ms = roof["ms"] if mixed["dom"] == "P2P" else other["ms"]

    def errs(res, pos_np, q_np, t_idx, phi_d, E_d):
        return sampled_errors(res, q_np, t_idx, phi_d, E_d)

    def mixed_vs_fp64(a_res, b_res, q_np):
        a, b = a_res["phi"].cpu().numpy(), b_res["phi"].cpu().numpy()
        Ea, Eb = a_res["E"].cpu().numpy(), b_res["E"].cpu().numpy()
        qq = q_np.astype(np.float64)[:, None]
        return {"phi": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                "F": float(np.linalg.norm(qq * (Ea - Eb)) / np.linalg.norm(qq * Eb))}

    # accuracy on sampled targets vs the FP64 direct sum
    t_idx = inputs.targets(n, wl.seed)
    phi_d, E_d = oracle.direct(pos_np.astype(np.float64), q_np.astype(np.float64), t_idx)
    rel = {"mixed_vs_direct": errs(mixed, pos_np, q_np, t_idx, phi_d, E_d)}
    fp64 = None
    if not args.no_fp64:
        fp64 = measure(fmm, wl, pos, q, "fp64", max(3, args.steps // 4), 1, sync)
        log("%s FP64 form measured" % args.workload)
        rel["fp64_vs_direct"] = errs(fp64, pos_np, q_np, t_idx, phi_d, E_d)
        rel["mixed_vs_fp64_all"] = mixed_vs_fp64(mixed, fp64, q_np)

    overlap = None
    if not args.no_overlap:
        ov = measure(fmm, wl, pos, q, "mixed", args.steps, args.warmup, sync, overlap_near=True, **enc_kw)
        overlap = {"ms_per_step": ov["sec"] * 1e3, "particles_per_s": n / ov["sec"],
                   "serial_ms_per_step": mixed["sec"] * 1e3,
                   "p2p_ms_side_stream": ov["stages_ms"]["P2P"], "m2l_ms": ov["stages_ms"]["M2L"]}
        del ov
        log("overlapped near field measured")

    c3 = None
    if not args.no_c3 and args.workload != "C3":
        w3 = inputs.WORKLOADS["C3"]
        p3, q3 = inputs.workload("C3")
        P3, Q3 = torch.from_numpy(p3).to(dev), torch.from_numpy(q3).to(dev)
        m3 = measure(fmm, w3, P3, Q3, "mixed", max(5, args.steps // 2), 2, sync, **enc_kw)
        log("C3 mixed form measured")
        r3, o3 = rooflines(w3, m3, "mixed", args.m2l, False)
        t3 = inputs.targets(w3.n, w3.seed)
        pd3, Ed3 = oracle.direct(p3, q3, t3)
        c3 = {"workload": w3.describe(), "levels": m3["info"]["levels"],
              "mixed": {"ms_per_step": m3["sec"] * 1e3, "particles_per_s": w3.n / m3["sec"],
                        "p2p_gint_s": m3["info"]["p2p_pairs"] / (m3["stages_ms"]["P2P"] * 1e-3) / 1e9,
                        "stages_ms": m3["stages_ms"], "roofline": r3,
                        ("roofline_p2p" if m3["dom"] == "M2L" else "roofline_m2l"): o3,
                        "tree_pass": tree_pass(w3, m3, "mixed")},
              "rel_l2": {"mixed_vs_direct": errs(m3, p3, q3, t3, pd3, Ed3)}}
        if not args.no_overlap:
            ov3 = measure(fmm, w3, P3, Q3, "mixed", max(5, args.steps // 2), 2, sync, overlap_near=True, **enc_kw)
            c3["overlap"] = {"ms_per_step": ov3["sec"] * 1e3, "particles_per_s": w3.n / ov3["sec"],
                             "p2p_ms_side_stream": ov3["stages_ms"]["P2P"], "m2l_ms": ov3["stages_ms"]["M2L"]}
            del ov3
            log("C3 overlapped near field measured")
        if not args.no_fp64:
            f3 = measure(fmm, w3, P3, Q3, "fp64", 3, 1, sync)
            log("C3 FP64 form measured")
            r3f, o3f = rooflines(w3, f3, "fp64", None, False)
            c3["fp64"] = {"ms_per_step": f3["sec"] * 1e3, "particles_per_s": w3.n / f3["sec"],
                          "p2p_gint_s": f3["info"]["p2p_pairs"] / (f3["stages_ms"]["P2P"] * 1e-3) / 1e9,
                          "stages_ms": f3["stages_ms"], "roofline": r3f}
            c3["rel_l2"]["fp64_vs_direct"] = errs(f3, p3, q3, t3, pd3, Ed3)
            c3["rel_l2"]["mixed_vs_fp64_all"] = mixed_vs_fp64(m3, f3, q3)
            del f3
        del m3, P3, Q3, p3, q3

    adj = None
    if not args.no_adjoint:
        w5 = inputs.WORKLOADS["C5"]
        p5, q5 = inputs.workload("C5")
        wv = torch.from_numpy(inputs.weights(w5.n, w5.seed)).to(dev)
        P5 = torch.from_numpy(p5).to(dev)
        Q5 = torch.from_numpy(q5).to(dev)
        tree5 = fmm.Tree(P5, p=w5.p, leaf_max=w5.leaf_max, precision="mixed", **enc_kw)

        def fb():
            tree5.rebuild(P5)
            _, E5 = tree5.evaluate(Q5)
            tree5.rebuild(P5)  # the tree is recomputed for the backward pass
            tree5.backward(Q5, wv, E5)

        s5 = timed_steps(fb, max(3, args.steps // 2), 2, sync)
        tree5.close()
        log("C5 forward + backward measured")
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
            t1 = fmm.Tree(P1, p=w1.p, leaf_max=w1.leaf_max, precision="mixed", **kw, **enc_kw)

            def ev():
                t1.evaluate(Q1, vec="field", phi=phi1, out_vec=E1)

            def st():
                t1.rebuild(P1)
                ev()

            small[name] = {"evaluate_us": 1e6 * timed_steps(ev, 200, 10, sync),
                           "step_us": 1e6 * timed_steps(st, 100, 5, sync)}
            t1.close()
        log("C1 launch modes measured")

    adaptive = None
    if not args.no_adaptive:
        adaptive = adaptive_record(fmm, oracle, inputs, max(5, args.steps // 2), 2, sync, dev,
                                   overlap=not args.no_overlap)
        log("adaptive tree measured")

    cpu = None
    if not args.no_cpu:
        ns = args.cpu_sample if args.cpu_sample > 0 else n
        ps, qs = inputs.particles(ns, wl.seed, wl.charges, wl.dtype)
        t0 = time.perf_counter()
        oracle.fmm(ps.astype(np.float64), qs.astype(np.float64), wl.p, wl.leaf_max)
        tc = time.perf_counter() - t0
        log("CPU oracle timed")
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
        "dtype": "f32+%s+f64" % args.m2l,
        "data": "synthetic",
        "config": {"workload": wl.describe(), "form": "mixed", "m2l_encoding": args.m2l,
                   "levels": info["levels"],
                   "p2p_pairs": pairs, "m2l_pairs": info["m2l_pairs"]},
        "p2p_gint_s": pairs / (p2p_ms * 1e-3) / 1e9,
        "stages_ms": mixed["stages_ms"],
        "roofline": roof,
        ("roofline_p2p" if mixed["dom"] == "M2L" else "roofline_m2l"): other,
        "tree_pass": tree_pass(wl, mixed, "mixed"),
        "tree_pass_c4_counters": tree_pass_counters(),
        "rel_l2": rel,
        "overlap": overlap,
        "c3": c3,
        "cpu_baseline": cpu,
        "adjoint": adj,
        "small": small,
        "adaptive": adaptive,
    }
    if fp64 is not None:
        r64, o64 = rooflines(wl, fp64, "fp64", None, False)
        line["fp64"] = {"particles_per_s": n / fp64["sec"], "ms_per_step": fp64["sec"] * 1e3,
                        "p2p_gint_s": pairs / (fp64["stages_ms"]["P2P"] * 1e-3) / 1e9,
                        "stages_ms": fp64["stages_ms"], "roofline": r64,
                        ("roofline_p2p" if fp64["dom"] == "M2L" else "roofline_m2l"): o64}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
