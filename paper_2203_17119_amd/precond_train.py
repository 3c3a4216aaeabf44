"""Train the gauge-equivariant preconditioner and measure what it gains in FGCR.

Recipe:
1. Training pairs.
   - On each of the ``8^4x8_train`` gauge fields (seeds 1100, 1101, ...), draw
     odd sources b~ and solve Mpc x = b~ with the library's own batched CG. The
     solve runs on the normal equations (Mpc^+ Mpc) x = Mpc^+ b~, in FP64, to a
     tolerance well below the loss the network can reach.
   - Sources: ``operator`` (default) takes b~ = Mpc v with Gaussian v. The
     solutions are then white, and the loss |N b~ - x|^2 / |x|^2 weighs every
     eigenmode of Mpc alike; it measures how far N Mpc is from the identity.
     ``gaussian`` takes Gaussian b~. Its solutions are dominated by the lowest
     modes, which a network of a few nearest-neighbour layers cannot represent.
   - Ten sources per field are held out for validation.
2. Training.
   - Adam on loss = mean |N(b~) - x|^2 / |x|^2, through ``dwf_net_train_step``: the
     network's own forward, backward and optimiser kernels.
   - Batches of 8 pairs from one field; the context's gauge field is switched
     with ``dwf_set_gauge``.
   - The network is a stack of parallel-transport convolutions (see
     ``include/dwf.h``), initialised to N = 1/d (the inverse of Mooee's diagonal)
     plus small noise.
3. Evaluation on ``24^4x12_fgcr``. Each solve is judged by its FP64 full residual:
   - plain FP64 CG, and the mixed FP16 CG;
   - plain GCR (no network);
   - FGCR with the initial network;
   - FGCR with the trained network.

``python -m paper_2203_17119_amd.precond_train --out weights.npz`` prints one
JSON line per phase and writes the trained weights.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import dwf, synth

CHANS = (4, 12, 12, 12, 4)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def init_weights(chans, d: float, seed: int, noise: float = 1e-3) -> np.ndarray:
    """Identity paths carrying the first channels through every layer, overall gain 1/d, plus noise."""
    rng = np.random.default_rng(seed)
    g = (1.0 / d) ** (1.0 / (len(chans) - 1))
    ws = []
    for ci, co in zip(chans[:-1], chans[1:]):
        w = noise * (rng.standard_normal((11, co, ci)) + 1j * rng.standard_normal((11, co, ci)))
        for a in range(min(ci, co)):
            w[0, a, a] += g
        ws.append(w.ravel())
    return np.concatenate(ws)


def make_pairs(lat, torch, gauges, per_field: int, seed0: int, tol: float = 1e-10, chunk: int = 50,
               sources: str = "operator"):
    """pairs[f] = list of (b~, x) device tensors on field f, x = Mpc^-1 b~ from the solver."""
    V = lat.V
    pairs = []
    for f, U in enumerate(gauges):
        dwf.dwf_set_gauge(lat.ctx, U)
        out = []
        for lo in range(0, per_field, chunk):
            n = min(chunk, per_field - lo)
            bs = [torch.from_numpy(synth.gaussian_fermion(lat.dims, lat.Ls, seed0 + 1000 * f + lo + k,
                                                          nsites=V // 2)).cuda() for k in range(n)]
            if sources == "operator":
                for k, v in enumerate(bs):
                    b = torch.empty_like(v)
                    dwf.dwf_schur_apply(lat.ctx, 0, v, b)
                    bs[k] = b
            elif sources != "gaussian":
                raise ValueError("sources must be 'operator' or 'gaussian'")
            rhs = [torch.empty_like(b) for b in bs]
            for b, r in zip(bs, rhs):
                dwf.dwf_schur_apply(lat.ctx, 1, b, r)
            xs = [torch.empty_like(b) for b in bs]
            status, st = dwf.dwf_multishift_cg(lat.ctx, rhs, [0.0], xs, tol=tol, mode=dwf.DWF_SOLVE_F64)
            if status != dwf.DWF_OK:
                raise RuntimeError(f"pair generation did not converge on field {f}")
            del rhs
            out.extend(zip(bs, xs))
        pairs.append(out)
    torch.cuda.synchronize()
    return pairs


def evaluate_loss(lat, net, gauges, pairs, batch: int = 8) -> float:
    tot, n = 0.0, 0
    for f, U in enumerate(gauges):
        if not pairs[f]:
            continue
        dwf.dwf_set_gauge(lat.ctx, U)
        ps = pairs[f]
        for lo in range(0, len(ps), batch):
            chunk = ps[lo:lo + batch]
            loss = dwf.dwf_net_train_step(net, [b for b, _ in chunk], [x for _, x in chunk], update=False)
            tot += loss * len(chunk)
            n += len(chunk)
    return tot / n


def train(lat, net, gauges, train_pairs, val_pairs, epochs: int, batch: int = 8, lr: float = 1e-3,
          seed: int = 0, every: int = 1):
    """Adam over the training pairs; returns the history [(epoch, train loss, validation loss, seconds)]."""
    rng = np.random.default_rng(seed)
    hist = [(0, evaluate_loss(lat, net, gauges, train_pairs), evaluate_loss(lat, net, gauges, val_pairs), 0.0)]
    log(f"epoch 0: train {hist[0][1]:.4f} val {hist[0][2]:.4f}")
    t0 = time.perf_counter()
    for ep in range(1, epochs + 1):
        batches = []
        for f in range(len(gauges)):
            idx = rng.permutation(len(train_pairs[f]))
            batches += [(f, idx[lo:lo + batch]) for lo in range(0, len(idx) - batch + 1, batch)]
        order = rng.permutation(len(batches))
        # group consecutive batches by field to limit gauge switches, in a random field order
        order = sorted(order, key=lambda k: (batches[k][0] * 7919 + ep * 104729) % len(gauges))
        cur = -1
        for k in order:
            f, idx = batches[k]
            if f != cur:
                dwf.dwf_set_gauge(lat.ctx, gauges[f])
                cur = f
            dwf.dwf_net_train_step(net, [train_pairs[f][i][0] for i in idx], [train_pairs[f][i][1] for i in idx],
                                   lr=lr)
        if ep % every == 0 or ep == epochs:
            tl = evaluate_loss(lat, net, gauges, train_pairs)
            vl = evaluate_loss(lat, net, gauges, val_pairs)
            hist.append((ep, tl, vl, time.perf_counter() - t0))
            log(f"epoch {ep}: train {tl:.4f} val {vl:.4f} ({time.perf_counter() - t0:.1f}s)")
    return hist


def solve_table(lat, torch, nets: dict, b_full, tol: float, restart: int, maxit: int, normal_too: bool = False,
                gcr: bool = True, mode: int = dwf.DWF_SOLVE_F64):
    """Time-to-tol of plain CG, plain GCR and FGCR with each network on one source
    (Schur system; with normal_too also the normal equations)."""
    rows = {}
    x = torch.zeros_like(b_full)
    torch.cuda.synchronize()
    s, st = dwf.dwf_cg(lat.ctx, b_full, x, tol=tol, mode=dwf.DWF_SOLVE_F64)
    rows["cg_f64"] = {"status": s, "iters": st["iters"], "seconds": st["seconds"], "res_full": st["res_full"]}
    x.zero_()
    s, st = dwf.dwf_cg(lat.ctx, b_full, x, tol=tol, mode=dwf.DWF_SOLVE_MIXED_F16)
    rows["cg_mixed_f16"] = {"status": s, "iters": st["iters"], "seconds": st["seconds"], "res_full": st["res_full"]}
    for normal in ((False, True) if normal_too else (False,)):
        tag = "normal" if normal else "schur"
        for name, net in ([("gcr", None)] if gcr else []) + list(nets.items()):
            x.zero_()
            dwf.dwf_kernel_timing_reset(lat.ctx)
            dwf.dwf_kernel_timing(lat.ctx, 1)
            s, st = dwf.dwf_fgcr(lat.ctx, net, b_full, x, tol=tol, restart=restart, normal=normal, maxit=maxit,
                                 fallback=False, mode=mode)
            kn = dwf.dwf_kernel_stats(lat.ctx, dwf.DWF_K_NET)
            dwf.dwf_kernel_timing(lat.ctx, 0)
            rows[f"{name}_{tag}"] = {"status": s, "iters": st["iters"], "seconds": st["seconds"],
                                     "res_full": st["res_full"], "net_ms": round(kn["ms"], 2),
                                     "net_launches": kn["launches"]}
            log(f"{name}_{tag}: {rows[f'{name}_{tag}']}")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fields", type=int, default=20)
    ap.add_argument("--per-field", type=int, default=100)
    ap.add_argument("--val-per-field", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--sources", default="operator", choices=("operator", "gaussian"))
    ap.add_argument("--out", default=None, help="write the trained weights (npz)")
    ap.add_argument("--weights", default=None, help="skip training: evaluate these weights (npz)")
    ap.add_argument("--eval-workload", default="24^4x12_fgcr")
    ap.add_argument("--eval-sources", type=int, default=1)
    ap.add_argument("--restart", type=int, default=32)
    ap.add_argument("--maxit", type=int, default=3000)
    ap.add_argument("--normal-too", action="store_true", help="also evaluate FGCR on the normal equations")
    ap.add_argument("--skip-init", action="store_true", help="do not evaluate the untrained network")
    ap.add_argument("--chans", default=",".join(map(str, CHANS)),
                    help="channel counts, comma separated (4 at both ends; 4, 8 or 12 each)")
    ap.add_argument("--skip-gcr", action="store_true", help="do not evaluate plain GCR")
    ap.add_argument("--mixed", action="store_true", help="FGCR with FP32 cycles and FP64 restarts")
    ap.add_argument("--bf16-basis", action="store_true",
                    help="FGCR with FP32 cycles, the Krylov basis in BF16 and FP64 restarts")
    ap.add_argument("--forward", default="both", choices=("both", "fp32", "mfma"),
                    help="network forward(s) to evaluate")
    args = ap.parse_args()

    import torch

    torch.cuda.set_device(0)
    if args.weights:
        data = np.load(args.weights)
        evaluate(args, torch, data["init"], data["weights"], tuple(int(v) for v in data["chans"]))
        return
    w = synth.WORKLOADS["8^4x8_train"]
    gauges = [torch.from_numpy(synth.gauge_field(w.dims, w.eps, w.gauge_seed + f)).cuda() for f in range(args.fields)]
    lat = dwf.Lattice(w.dims, w.Ls, w.b, w.c, w.M5, w.mf, w.dirichlet, gauge=gauges[0])
    d = w.b * (4 - w.M5) + 1
    t0 = time.perf_counter()
    pairs = make_pairs(lat, torch, gauges, args.per_field, seed0=3_000_000, sources=args.sources)
    t_pairs = time.perf_counter() - t0
    nval = args.val_per_field
    train_pairs = [p[:-nval] for p in pairs]
    val_pairs = [p[-nval:] for p in pairs]
    log(f"{sum(map(len, pairs))} pairs in {t_pairs:.1f}s")
    chans = tuple(int(v) for v in args.chans.split(","))
    net = dwf.dwf_net_create(lat.ctx, chans)
    w0 = init_weights(chans, d, seed=5)
    dwf.dwf_net_set_weights(net, w0)
    hist = train(lat, net, gauges, train_pairs, val_pairs, args.epochs, lr=args.lr)
    wt = dwf.dwf_net_get_weights(net)
    dwf.dwf_net_destroy(net)
    lat.close()
    print(json.dumps({"phase": "train", "lattice": "8^4x8", "fields": args.fields, "sources": args.sources,
                      "chans": list(chans),
                      "pairs": sum(map(len, pairs)), "pair_seconds": round(t_pairs, 2),
                      "history": [[e, round(a, 5), round(b, 5), round(s, 2)] for e, a, b, s in hist]}), flush=True)
    if args.out:
        np.savez(args.out, weights=wt, chans=np.array(chans), init=w0)

    evaluate(args, torch, w0, wt, chans)


def evaluate(args, torch, w0, wt, chans=CHANS):
    ev = synth.WORKLOADS[args.eval_workload]
    U = synth.gauge_field(ev.dims, ev.eps, ev.gauge_seed)
    lat = dwf.Lattice(ev.dims, ev.Ls, ev.b, ev.c, ev.M5, ev.mf, ev.dirichlet, gauge=U)
    del U
    nets = {}
    for name, wts in (("net_init", w0), ("net_trained", wt), ("net_trained_mfma", wt)):
        if name == "net_init" and args.skip_init:
            continue
        if (name.endswith("_mfma") and args.forward == "fp32") or (name == "net_trained" and args.forward == "mfma"):
            continue
        nets[name] = dwf.dwf_net_create(lat.ctx, chans)
        dwf.dwf_net_set_weights(nets[name], wts)
        if name.endswith("_mfma"):
            dwf.dwf_net_set_forward(nets[name], dwf.DWF_NET_FWD_MFMA_BF16)
    for k in range(args.eval_sources):
        b = torch.from_numpy(synth.gaussian_fermion(ev.dims, ev.Ls, ev.source_seeds[k])).cuda()
        rows = solve_table(lat, torch, nets, b, ev.tol, args.restart, args.maxit, args.normal_too, not args.skip_gcr,
                           dwf.DWF_SOLVE_MIXED_BF16 if args.bf16_basis
                           else dwf.DWF_SOLVE_MIXED_F32 if args.mixed else dwf.DWF_SOLVE_F64)
        print(json.dumps({"phase": "eval", "workload": args.eval_workload, "source": ev.source_seeds[k],
                          "restart": args.restart, "rows": rows}), flush=True)
    for n in nets.values():
        dwf.dwf_net_destroy(n)
    lat.close()


if __name__ == "__main__":
    main()
