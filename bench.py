#!/usr/bin/env python3
"""End-to-end benchmark of the RaftGP hot path on one MI355X.

One step = the whole path on one synthetic graph already resident in HBM:
graph ingest (CSR validation and degrees from the device-resident CSR), then
for each projection variant (NCut and full modularity by default) the random
projection, the random GCN, k-means over every candidate K, the per-edge
scores and the selection of K*.  `value` is graphs per second (both variants
per graph).

The dominant kernel class is timed live with HIP events around each of its
launches inside the timed steps (library profiling hooks); its algorithmic
work per launch gives the roofline fraction.  The FP64 oracle is timed on a
bounded sample of the same workload on the host cores (rank 0, N=1 only).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload n50k|n1m]
"""
import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12            # bytes/s, MI355X HBM3E
PEAK_MFMA_F32 = 157.3e12     # FLOP/s, dense FP32 matrix
PEAK_MFMA_F16 = 2.5e15       # FLOP/s, dense FP16 matrix
VARIANTS = {"ncut": 0, "mod_full": 1, "mod_reduced": 2}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="n50k")
    ap.add_argument("--variants", default="ncut,mod_full")
    ap.add_argument("--concurrent-variants", action="store_true",
                    help="time the steps with each variant on its own context and stream, "
                         "driven from its own host thread, so their kernels overlap (default: "
                         "one after the other on one stream; the overlapped schedule is then "
                         "timed as an extra record unless --no-extras)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-stride", type=int, default=26)
    ap.add_argument("--train", action="store_true",
                    help="time the trainable-GCN mode on the n200k workload instead")
    ap.add_argument("--train-steps", type=int, default=200)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-vs-sequential leg")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sampler (Alg. 2) and streaming (Sec. III-D) records")
    ap.add_argument("--batch-graphs", type=int, default=64)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "assign": ["paper_2312_01560_amd/csrc/kmeans.hip"],  # k_assign / k_assign_h
    "spmm": ["paper_2312_01560_amd/csrc/spmm.hip"],
    "score": ["paper_2312_01560_amd/csrc/score.hip"],
}


def measured_traffic(kind, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None if
    absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(f"{kind}:{workload}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != source_hash(KERNEL_SOURCES[kind]):
        return None
    return rec.get("bytes_per_launch")


def host_description():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"os_cpu_count": os.cpu_count(), "cpu_model": model}


def cpu_baseline(graph, method, variants, gpu_out, stride):
    """The FP64 oracle, as it stands, on a bounded sample of one step: the
    whole projection and GCN of every variant; the oracle's own k-means++
    seeding to the largest sampled K; its own Lloyd and scores for every
    `stride`-th candidate plus the GPU's K*, each timed alone.  The grid's
    k-means time is estimated from the oracle's own per-candidate times,
    interpolated linearly in K between the sampled candidates, and the
    seeding time scaled to K_max (one race step per pick)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import gcn, kmeans, projection, scores

    ks = list(range(method["k_min"], method["k_max"] + 1, method["k_step"]))
    total_s = 0.0
    sampled_s = 0.0
    nmis = []
    nmi_star = []
    sample_desc = []
    for name in variants:
        op = VARIANTS[name]
        t0 = time.perf_counter()
        y = projection.project(graph.row_ptr, graph.col_idx, graph.n, op, method["proj_dim"],
                               method["q"], 0)
        z = gcn.embed(graph.row_ptr, graph.col_idx, graph.n, y, method["layer_dims"], 0)
        t_embed = time.perf_counter() - t0
        out = gpu_out[name]
        best = int(out["k_selected"][2])
        sample = sorted(set(range(0, len(ks), stride)) | {best, len(ks) - 1})
        kseed = max(ks[j] for j in sample)
        t0 = time.perf_counter()
        picks = kmeans.seed_picks(z, kseed, 0)
        t_seed = time.perf_counter() - t0
        per = {}
        labs = {}
        for j in sample:
            t0 = time.perf_counter()
            a, _, _ = kmeans.lloyd(z, z[picks[:ks[j]]], 100)
            scores.modularity(graph.row_ptr, graph.col_idx, a, ks[j])
            scores.ncut(graph.row_ptr, graph.col_idx, a, ks[j])
            per[j] = time.perf_counter() - t0
            labs[j] = a
        xs = [ks[j] for j in sample]
        grid_km = float(np.sum(np.interp(ks, xs, [per[j] for j in sample])))
        est = t_embed + t_seed * max(ks) / kseed + grid_km
        total_s += est
        sampled_s += t_embed + t_seed + sum(per.values())
        for j in sample:
            v = scores.nmi(out["labels_all"][:, j], labs[j])
            nmis.append(v)
            if j == best:
                nmi_star.append(v)
        sample_desc.append(f"{name}: projection+GCN {t_embed:.1f} s (whole), seeding to K={kseed} "
                           f"{t_seed:.1f} s, Lloyd+scores for K in {xs} "
                           f"({sum(per.values()):.1f} s), grid estimate {est:.1f} s")
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    host = host_description()
    return {
        "value": 1.0 / total_s, "unit": "graphs/s", "cores": threads, "kind": "oracle",
        "sample": "; ".join(sample_desc) + f"; {sampled_s:.1f} s of oracle work timed; "
                  f"estimated {total_s:.1f} s per graph (both variants); BLAS threads "
                  f"{threads} on {host['os_cpu_count']} logical CPUs ({host['cpu_model']}); "
                  "scipy.sparse products single-threaded",
        "seconds": total_s, "host": host,
    }, float(min(nmis)), float(min(nmi_star))


def bench_train(args, api, torch, np):
    """Trainable-weight GCN on the n200k workload: 3 layers of width 64, the
    last one linear into 64 softmax assignments, loss -tr(S^T B S)/2e, Adam.
    One step = forward + loss + adjoint + Adam on every W (activations are
    recomputed in the adjoint).  The untrained start is the method's own random
    GCN; both are compared with the method's partition by modularity and NMI."""
    from paper_2312_01560_amd.train import Trainer
    from synth import make_workload
    graph, method = make_workload("n200k")
    ctx = api.Context(0)
    dev = ctx.torch_device
    g = api.Graph(ctx, torch.from_numpy(graph.row_ptr).to(dev), torch.from_numpy(graph.col_idx).to(dev))
    dims = [64, 64, 64, 64]
    cfg = api.Config(op=1, proj_dim=64, q=3, layer_dims=dims[1:], k_min=2, k_max=64)
    log(f"n200k: n={graph.n} nnz={graph.nnz}; method run (untrained random GCN)")
    base = api.run(ctx, g, cfg)
    torch.cuda.synchronize()
    y = base["Y"]
    ws = [api.gaussian(ctx, cfg.seed, api.STREAM_W_BASE + k + 1, dims[k], dims[k + 1],
                       1.0 / np.sqrt(dims[k])) for k in range(3)]
    tr = Trainer(ctx, g, dims)
    params = [w.clone() for w in ws]
    ms = [torch.zeros_like(w) for w in ws]
    vs = [torch.zeros_like(w) for w in ws]

    def nmi_dev(a, b):
        return api.nmi(ctx, torch.from_numpy(np.asarray(a, dtype=np.int32)).to(dev),
                       torch.from_numpy(np.asarray(b, dtype=np.int32)).to(dev))

    def hard(S):
        lab = torch.argmax(S, dim=1).to(torch.uint8)[:, None].contiguous()
        mod, _ = api.score(ctx, g, lab, [64])
        return lab[:, 0].cpu().numpy().astype(np.int64), float(mod.cpu()[0])

    U, _ = tr.forward(y, params)
    S0, loss0 = tr.modloss_forward(U)
    lab0, mod0 = hard(S0)
    losses = [float(loss0.cpu()[0])]
    log(f"training {args.train_steps} Adam steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(1, args.train_steps + 1):
        U, saved = tr.forward(y, params)
        S, loss = tr.modloss_forward(U)
        GW, _ = tr.backward(y, params, saved, tr.modloss_backward(S))
        for k in range(3):
            tr.adam(params[k], ms[k], vs[k], GW[k], step)
        if step % 50 == 0:
            losses.append(float(loss.cpu()[0]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync_status()
    U, _ = tr.forward(y, params)
    S1, loss1 = tr.modloss_forward(U)
    lab1, mod1 = hard(S1)
    method_lab = base["labels"].cpu().numpy()
    method_mod = float(base["mod"].cpu().numpy()[int(base["k_selected"].cpu()[2])])
    ms_step = 1e3 * (t1 - t0) / args.train_steps
    rec = {
        "metric": "trainable GCN steps/s (forward + relaxed-modularity loss + adjoint + Adam), n200k",
        "value": 1e3 / ms_step, "unit": "steps/s", "n_gpus": 1, "steps": args.train_steps,
        "warmup": 0, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "n200k", "n": graph.n, "nnz": graph.nnz, "dims": dims,
                   "softmax_k": 64, "optimizer": "adam lr 1e-2"},
        "loss": {"step0": losses[0], "every50": losses[1:], "final": float(loss1.cpu()[0])},
        "modularity": {"untrained_softmax_argmax": mod0, "trained_softmax_argmax": mod1,
                       "method_partition": method_mod},
        "nmi": {"trained_vs_untrained": nmi_dev(lab1, lab0),
                "trained_vs_method": nmi_dev(lab1, method_lab),
                "trained_vs_planted": nmi_dev(lab1, graph.planted),
                "method_vs_planted": nmi_dev(method_lab, graph.planted)},
        "spmm_per_step": 9,
    }
    print(json.dumps(rec))
    ctx.close()


def bench_sampler(api, torch, np, ctx):
    """Alg. 2 on the device: DC-SBM models of 50k nodes / 44 blocks (the
    n50k recipe) and 1M nodes / 100 blocks (the n1m recipe), sampled into a
    validated graph; best of three calls, host preparation included."""
    from synth.dcsbm import dcsbm_model
    out = {}
    for name, n, k, dmax, gamma in (("n50k", 50000, 44, 300.0, 2.5),
                                    ("n1m", 1000000, 100, 1000.0, 2.3)):
        theta, blocks, omega = dcsbm_model(n, k, gamma=gamma, d_max=dmax, rho=2.0, seed=7)
        api.sbm_sample(ctx, theta, blocks, omega, 0).close()
        best, edges = 1e9, 0
        for rep in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g = api.sbm_sample(ctx, theta, blocks, omega, rep + 1)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
            edges = g.nnz // 2
            g.close()
        out[name] = {"n": n, "blocks": k, "edges": int(edges), "ms": round(best * 1e3, 3),
                     "edges_per_s": edges / best}
    return out


def bench_stream(api, torch, np, ctx, graph, method):
    """Streaming update (Sec. III-D) on the n50k graph, NCut: 64 random new
    edges added to a stream against a full projection + GCN of the new
    graph; and the same for a shallow configuration (q = 1, one layer),
    whose hop balls stay small."""
    out = {}
    rng = np.random.default_rng(11)
    n = graph.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(graph.row_ptr))
    have = set((rows * n + graph.col_idx.astype(np.int64)).tolist())
    for name, upd in (("q3_gcn2", {}), ("q1_gcn1", {"q": 1, "layer_dims": method["layer_dims"][:1]})):
        m = dict(method)
        m.update(upd)
        cfg = api.Config(op=api.X_NCUT, seed=0, **m)
        g = api.Graph(ctx, graph.row_ptr, graph.col_idx)
        ws = ctx.workspace(api.workspace_size(ctx, g, cfg))
        for _ in range(2):
            api.embed(ctx, g, cfg, api.project(ctx, g, cfg, ws=ws), ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            api.embed(ctx, g, cfg, api.project(ctx, g, cfg, ws=ws), ws=ws)
        torch.cuda.synchronize()
        full = (time.perf_counter() - t0) / 5
        st = api.Stream(ctx, g, cfg)
        times, balls = [], None
        for rep in range(4):
            e = set()
            while len(e) < 64:
                a, b = (int(v) for v in rng.integers(0, n, 2))
                a, b = min(a, b), max(a, b)
                if a != b and a * n + b not in have and (a, b) not in e:
                    e.add((a, b))
            for a, b in e:
                have.add(a * n + b)
                have.add(b * n + a)
            src = np.array([a for a, _ in e]), np.array([b for _, b in e])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            balls = st.add_edges(*src)
            torch.cuda.synchronize()
            if rep > 0:
                times.append(time.perf_counter() - t0)
        st.close()
        g.close()
        out[name] = {"new_edges": 64, "update_ms": round(1e3 * min(times), 3),
                     "full_reembed_ms": round(1e3 * full, 3),
                     "rows_per_level": [int(x) for x in balls]}
    # a 1M-node graph sampled on the device (the n1m model), L = 128, q = 1,
    # one 128-wide layer; 1 and 16 new edges
    from synth.dcsbm import dcsbm_model
    theta, blocks, omega = dcsbm_model(1000000, 100, gamma=2.3, d_max=1000.0, rho=2.0, seed=7)
    g = api.sbm_sample(ctx, theta, blocks, omega, 1)
    cfg = api.Config(op=api.X_NCUT, proj_dim=128, q=1, layer_dims=[128], k_min=50, k_max=150,
                     k_step=5, seed=0)
    ws = ctx.workspace(api.workspace_size(ctx, g, cfg))
    api.embed(ctx, g, cfg, api.project(ctx, g, cfg, ws=ws), ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        api.embed(ctx, g, cfg, api.project(ctx, g, cfg, ws=ws), ws=ws)
    torch.cuda.synchronize()
    full = (time.perf_counter() - t0) / 3
    del ws
    st = api.Stream(ctx, g, cfg)
    grp, gci = (t.cpu().numpy() for t in g.csr())
    g.close()
    n = 1000000
    added = set()

    def present(a, b):
        row = gci[grp[a]:grp[a + 1]]
        k = int(np.searchsorted(row, b))
        return (k < row.size and row[k] == b) or (a, b) in added

    res = {}
    for m in (1, 1, 16, 16):
        e = set()
        while len(e) < m:
            a, b = (int(v) for v in rng.integers(0, n, 2))
            a, b = min(a, b), max(a, b)
            if a != b and not present(a, b) and (a, b) not in e:
                e.add((a, b))
        added |= e
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        balls = st.add_edges(np.array([a for a, _ in e]), np.array([b for _, b in e]))
        torch.cuda.synchronize()
        res[m] = (time.perf_counter() - t0, [int(x) for x in balls])   # second of each size kept
    st.close()
    out["n1m_q1_gcn1"] = {"full_reembed_ms": round(1e3 * full, 3),
                          "updates": {str(m): {"update_ms": round(1e3 * t, 3), "rows_per_level": b}
                                      for m, (t, b) in res.items()}}
    return out


def bench_batch(args, api, torch, np, ctx):
    """The batched workload: 64 DC-SBM graphs (N log-uniform on [1e3, 5e4])
    through the whole path (modularity variant, K 2..64) as one batch -- one
    block-diagonal CSR, one launch per stage over all graphs and candidates,
    the fixed prefix replayed from a HIP graph -- against the same graphs run
    one at a time through the single-graph calls.  Both legs start from
    ingested graphs, preallocated outputs and workspaces; per-graph labels of
    the two legs are compared (NMI) and against the planted blocks."""
    from synth.workloads import make_batch
    graphs, method = make_batch(args.batch_graphs)
    dev = ctx.torch_device
    cfg = api.Config(op=1, **method)
    gs = [api.Graph(ctx, torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col_idx).to(dev))
          for g in graphs]
    b = api.Batch(ctx, gs, cfg)
    bouts = b.outputs()
    log(f"batch: {len(graphs)} graphs, N={sum(g.n for g in graphs)}, "
        f"nnz={sum(g.nnz for g in graphs)}; warm-up")
    for _ in range(max(1, args.warmup // 2)):
        b.run(outputs=bouts)
    torch.cuda.synchronize()
    reps = max(1, args.batch_reps)
    t0 = time.perf_counter()
    for _ in range(reps):
        b.run(outputs=bouts)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    stages = b.stage_times()
    ws = ctx.workspace(max(api.workspace_size(ctx, g, cfg) for g in gs))
    souts = [api._outputs(ctx, g, cfg) for g in gs]
    for g, o in zip(gs, souts):                      # warm-up of the sequential leg
        api.run(ctx, g, cfg, ws=ws, outputs=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for g, o in zip(gs, souts):
            api.run(ctx, g, cfg, ws=ws, outputs=o)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / reps
    ctx.sync_status()
    bres = [o for o, _ in bouts]
    same = sum(int(torch.equal(bo["labels"], so[0]["labels"]) and
                   torch.equal(bo["labels_all"], so[0]["labels_all"]))
               for bo, so in zip(bres, souts))
    nmi_bs = [api.nmi(ctx, bo["labels"], so[0]["labels"]) for bo, so in zip(bres, souts)]
    nmi_pl = [api.nmi(ctx, bo["labels"], torch.from_numpy(g.planted.astype(np.int32)).to(dev))
              for bo, g in zip(bres, graphs)]
    tune_factor, tune_ms = b.tuning()
    b.close()
    for g in gs:
        g.close()
    return {
        "workload": f"batch{len(graphs)}: {len(graphs)} DC-SBM graphs, N log-uniform on "
                    "[1e3, 5e4], modularity variant, K 2..64",
        "graphs": len(graphs), "n_total": int(sum(g.n for g in graphs)),
        "nnz_total": int(sum(g.nnz for g in graphs)),
        "batched_graphs_per_s": len(graphs) / t_batch,
        "sequential_graphs_per_s": len(graphs) / t_seq,
        "speedup": t_seq / t_batch,
        "ms_per_batch": 1e3 * t_batch, "ms_sequential": 1e3 * t_seq, "reps": reps,
        "batch_stage_ms": dict(zip(["prefix", "lloyd", "score"], [round(v, 3) for v in stages])),
        "autotune": {"share_factor": tune_factor,
                     "candidates_ms": {str(f): round(t, 3) for f, t in tune_ms},
                     "note": "per-graph result-invariant shapes (update ranges, edge-score and "
                             "race grids) sized for CU share = num_cu x factor x n_g / N "
                             "(0 = single-graph shapes); first run times each candidate"},
        "graphs_bit_identical_to_sequential": same,
        "nmi_batched_vs_sequential_min": float(min(nmi_bs)),
        "nmi_vs_planted_mean": float(np.mean(nmi_pl)),
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the hot path is single-GPU; "
              "multi-GPU sharding is a design note only", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2312_01560_amd import api
    from synth import make_workload

    if args.train:
        bench_train(args, api, torch, np)
        return
    if args.workload not in ("n50k", "n1m", "small", "n200k"):
        print(f"unknown workload {args.workload}", file=sys.stderr)
        sys.exit(2)
    graph, method = make_workload(args.workload)
    variants = [v for v in args.variants.split(",") if v]
    ctx = api.Context(0)
    dev = ctx.torch_device
    rp = torch.from_numpy(graph.row_ptr).to(dev)
    ci = torch.from_numpy(graph.col_idx).to(dev)
    cfgs = {v: api.Config(op=VARIANTS[v], **method) for v in variants}
    # The variants of a step are independent runs over the same graph.  By
    # default each has its own context (workspace, events, pinned staging)
    # and stream and is driven from its own host thread, so the kernels of
    # one fill the latency of the other's; every result is the same as in a
    # serial run.  Streams keep the default priority.
    concurrent = len(variants) > 1 and args.concurrent_variants
    conc_leg = len(variants) > 1 and not concurrent and not args.no_extras
    two = concurrent or conc_leg
    vctx = {v: (api.Context(0) if two and i > 0 else ctx) for i, v in enumerate(variants)}
    vstream = {v: torch.cuda.Stream() for v in variants} if two else {}
    ctxs = list({id(c): c for c in vctx.values()}.values())
    wsv, outs = {}, {}
    for v in variants:
        c = vctx[v]
        g0 = api.Graph(c, rp, ci)
        if two:
            wsv[v] = c.workspace(api.workspace_size(c, g0, cfgs[v]))
        elif variants[0] in wsv:
            wsv[v] = wsv[variants[0]]
        else:
            wsv[v] = ctx.workspace(max(api.workspace_size(ctx, g0, cf) for cf in cfgs.values()))
        outs[v] = api._outputs(c, g0, cfgs[v], want_y=True, want_z=True)
        g0.close()

    def steps(k, acc=None, conc=concurrent):
        """k steps: every variant over a graph created for the step."""
        if not conc:
            for _ in range(k):
                g = api.Graph(ctx, rp, ci)
                for v in variants:
                    api.run(ctx, g, cfgs[v], ws=wsv[v], outputs=outs[v])
                    if acc is not None:
                        acc[v] += np.array(api.stage_times(ctx))
                g.close()
            return
        errors = []

        def worker(v):
            try:
                c = vctx[v]
                with torch.cuda.stream(vstream[v]):
                    for _ in range(k):
                        g = api.Graph(c, rp, ci)
                        api.run(c, g, cfgs[v], ws=wsv[v], outputs=outs[v])
                        if acc is not None:
                            acc[v] += np.array(api.stage_times(c))
                        g.close()
                    vstream[v].synchronize()
            except BaseException as e:   # re-raised in the main thread
                errors.append(e)

        threads = [threading.Thread(target=worker, args=(v,)) for v in variants]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if errors:
            raise errors[0]

    log(f"workload {args.workload}: n={graph.n} nnz={graph.nnz} variants={variants} "
        f"({'concurrent' if concurrent else 'serial'}); warm-up")
    steps(args.warmup)
    torch.cuda.synchronize()
    for c in ctxs:
        c.sync_status()
    log("warm-up done; timed steps")
    for c in ctxs:
        api.profile_read(c)
        api.profile_enable(c, (1 << 0) | (1 << 3) | (1 << 5))   # SpMM, assignment, edge scores
    stage = {v: np.zeros(5) for v in variants}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps(args.steps, stage)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {}
    for c in ctxs:
        for key, (ms, cnt) in api.profile_read(c).items():
            m0, c0 = prof.get(key, (0.0, 0))
            prof[key] = (m0 + ms, c0 + cnt)
        api.profile_enable(c, 0)
        c.sync_status()
    conc_rec = None
    if conc_leg:
        # the same steps with the variants overlapped (after one untimed step)
        lab_serial = {v: outs[v][0]["labels_all"].clone() for v in variants}
        steps(1, conc=True)
        torch.cuda.synchronize()
        tc0 = time.perf_counter()
        steps(args.steps, conc=True)
        torch.cuda.synchronize()
        tc = time.perf_counter() - tc0
        for c in ctxs:
            c.sync_status()
        conc_rec = {"value": args.steps / tc, "unit": "graphs/s",
                    "ms_per_step": 1e3 * tc / args.steps,
                    "schedule": "a context, stream and host thread per variant",
                    "labels_identical_to_serial": all(
                        bool(torch.equal(lab_serial[v], outs[v][0]["labels_all"]))
                        for v in variants)}
        log(f"variants overlapped: {conc_rec['ms_per_step']:.2f} ms/step")
    elapsed = t1 - t0
    log(f"timed steps done: {1e3 * elapsed / args.steps:.2f} ms/step")
    value = args.steps / elapsed

    host = {v: {k: t.cpu().numpy() for k, t in outs[v][0].items()} for v in variants}
    n, nnz = graph.n, graph.nnz
    d = cfgs[variants[0]].embed_dim
    ks = cfgs[variants[0]].ks
    # algorithmic work of one step
    assign_flops = sum(2.0 * n * d * float(np.dot(ks, host[v]["iters"])) for v in variants)
    kpad = [(k + 15) // 16 * 16 for k in ks]
    issued_flops = sum(3 * 2.0 * n * d * float(np.dot(kpad, host[v]["iters"])) for v in variants)
    spmm_bytes_per_launch = 4.0 * (n + 1) + 4.0 * nnz + 8.0 * n * method["proj_dim"]
    ms_assign, n_assign = prof["assign"]
    ms_spmm, n_spmm = prof["spmm"]
    ms_score, n_score = prof["score"]
    # edge scores: row pointers, column indices, one label row per node, the
    # row order (the neighbour label gathers are the same rows again)
    score_bytes_per_launch = 4.0 * (n + 1) + 4.0 * nnz + float(n) * len(ks) + 4.0 * n
    score_ach = score_bytes_per_launch * n_score / (ms_score * 1e-3) if ms_score > 0 else 0.0
    assign_ach = assign_flops * args.steps / (ms_assign * 1e-3) if ms_assign > 0 else 0.0
    spmm_ach = spmm_bytes_per_launch * n_spmm / (ms_spmm * 1e-3) if ms_spmm > 0 else 0.0
    dominant = "assign" if ms_assign >= ms_spmm else "spmm"
    pruned = False
    if dominant == "assign":
        split = d % 32 == 0
        peak = PEAK_MFMA_F16 if split else PEAK_MFMA_F32
        kname = ("k_assign_h (operands as split fp16 halves: three fp16 MFMA products per FP32 "
                 "product, FP32 accumulate)") if split else "k_assign (MFMA FP32)"
        roof = {"kernel": kname, "bound": "mfma",
                "achieved": assign_ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": assign_ach / peak,
                "flops_counted": "the method's 2 N d sum(K) per Lloyd iteration over the "
                                 "candidates still iterating",
                "per_launch": {"flops": assign_flops * args.steps / max(n_assign, 1),
                               "avg_ms": ms_assign / max(n_assign, 1)}}
        pruned = split and cfgs[variants[0]].kmeans_prune != 2 and (
            cfgs[variants[0]].kmeans_prune == 1 or float(np.mean(ks)) >= 64)
        if split and not pruned:
            # what the matrix unit actually executes: three fp16 products per
            # FP32 product, centre rows padded to multiples of 16
            issued = issued_flops * args.steps / (ms_assign * 1e-3) if ms_assign > 0 else 0.0
            roof["issued_mfma"] = {"achieved": issued / 1e12, "frac": issued / PEAK_MFMA_F16,
                                   "note": "3 fp16 products per FP32 product, padded centres"}
        if pruned:
            roof["kernel"] = ("bound-pruned assignment (k_prune_test + k_prune_score, the "
                              "first two iterations k_assign_h)")
            roof["note"] = ("a launch is one iteration's assignment; from the third on only the "
                            "points whose bounds do not hold their label are scored, so the "
                            "rate on the method's full Lloyd FLOPs is an effective one")
    else:
        roof = {"kernel": "k_spmm", "bound": "hbm", "achieved": spmm_ach / 1e9,
                "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": spmm_ach / PEAK_HBM,
                "per_launch": {"bytes": spmm_bytes_per_launch, "avg_ms": ms_spmm / max(n_spmm, 1)}}
    if concurrent:
        roof["duration_note"] = ("launch durations timed while the other variant's kernels "
                                 "share the GPU (the variants run concurrently), so the "
                                 "per-launch rate is below that of a kernel running alone")
    roof["traffic"] = measured_traffic(dominant, args.workload)
    if dominant == "assign" and pruned:
        roof["traffic"] = None   # the counters cover the full assignment kernel only
    roof["traffic_note"] = ("bytes per launch beyond L2 from two rocprofv3 counter passes "
                            "(FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, scaled by a plain copy): "
                            "Infinity Cache hits included, so an upper bound on HBM bytes; "
                            "null once the kernel source differs from the profiled one")

    planted = torch.from_numpy(graph.planted.astype(np.int32)).to(dev)
    nmi_planted = {v: api.nmi(ctx, outs[v][0]["labels"], planted) for v in variants}

    rec = {
        "metric": "end-to-end graphs/s (N=50k DC-SBM, NCut + modularity variants), "
                  "SpMM GB/s (% HBM peak), NMI vs oracle",
        "value": value, "unit": "graphs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (k-means distances: split-fp16 x3 MFMA, FP32 accumulate; FP64 reductions)",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "nnz": nnz, "edges": nnz // 2,
                   "proj_dim": method["proj_dim"], "q": method["q"],
                   "layer_dims": method["layer_dims"],
                   "k_grid": [method["k_min"], method["k_max"], method["k_step"]],
                   "variants": variants,
                   "variant_schedule": ("concurrent: a context, stream and host thread per "
                                        "variant" if concurrent else "serial: one stream")},
        "roofline": roof,
        "variants_concurrent": conc_rec,
        "spmm": {"achieved_gbs": spmm_ach / 1e9, "frac_hbm": spmm_ach / PEAK_HBM,
                 "avg_us": 1e3 * ms_spmm / max(n_spmm, 1), "launches": n_spmm,
                 "bytes_per_launch": spmm_bytes_per_launch,
                 "edges_features_per_s": nnz * method["proj_dim"] * n_spmm / (ms_spmm * 1e-3)
                 if ms_spmm > 0 else 0.0,
                 "traffic": measured_traffic("spmm", args.workload)},
        "edge_score": {"achieved_gbs": score_ach / 1e9, "frac_hbm": score_ach / PEAK_HBM,
                       "avg_us": 1e3 * ms_score / max(n_score, 1), "launches": n_score,
                       "bytes_per_launch": score_bytes_per_launch,
                       "edge_candidates_per_s": nnz * len(ks) * n_score / (ms_score * 1e-3)
                       if ms_score > 0 else 0.0,
                       "traffic": measured_traffic("score", args.workload)},
        "stages_ms_per_step": {v: dict(zip(["project", "embed", "seed", "lloyd", "score"],
                                           (stage[v] / args.steps).round(3).tolist()))
                               for v in variants},
        "k_star": {v: int(host[v]["k_selected"][0]) for v in variants},
        "nmi_vs_planted": nmi_planted,
    }
    if not args.no_batch and args.workload == "n50k":
        log("batched workload (batched vs one graph at a time)")
        rec["batch"] = bench_batch(args, api, torch, np, ctx)
    if not args.no_extras and args.workload == "n50k":
        log("sampler (Alg. 2) and streaming update (Sec. III-D) records")
        rec["sampler"] = bench_sampler(api, torch, np, ctx)
        rec["stream"] = bench_stream(api, torch, np, ctx, graph, method)
    if args.copy_calib_mib:
        a = torch.empty(args.copy_calib_mib << 18, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        rec["copy_calib_bytes"] = a.numel() * 4
    if not args.no_cpu_baseline:
        log("oracle on the host (cpu_baseline sample)")
        base, nmi_min, nmi_star = cpu_baseline(graph, method, variants, host,
                                               args.cpu_sample_stride)
        rec["cpu_baseline"] = base
        rec["nmi_vs_oracle"] = {"selected_k": nmi_star, "min_over_sample": nmi_min}
    print(json.dumps(rec))
    ctx.close()


if __name__ == "__main__":
    main()
