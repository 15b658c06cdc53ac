"""Benchmark of the whole hot path on one MI355X.

One step = one pass over every hot-path step at full size:
  * packed EDM, n = 65,536, d = 64, FP32 difference form, lambda2 map;
  * packed EDM via the Gram form, n = 32,768, d = 512, split BF16 on MFMA,
    lambda2 map;
  * Axilrod-Teller + Lennard-Jones energy and gradient (forward + backward),
    n = 8,192 RSA particles, lambda3 map (triplets) and lambda2 map (pairs).
The metric is simplex elements per second over the step (pairs of both EDMs,
triplets, LJ pairs).  Inputs are synthetic (seeded), resident in HBM before the
timed region.  Kernel durations come from HIP events the library records on
the launch stream; bounding-box and linear-map runs of the same steps are timed
after the main loop for the lambda-vs-bounding-box comparison.  The oracle is
timed on a bounded sample on the host cores (cpu_baseline).

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-compare]
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

# published MI355X peaks
PEAK_HBM = 8.0e12          # B/s
PEAK_FP32 = 157.3e12       # FLOP/s, vector FP32 (packed); 78.6e12 without packed FP32
PEAK_BF16 = 2.5e15         # FLOP/s, dense MFMA
AT_FLOPS_FWD, AT_FLOPS_FWD_BWD = 20, 80   # declared flops per triplet
LJ_FLOPS = 30                              # declared flops per pair (fwd + bwd)

# HBM bytes per launch of the Axilrod-Teller gradient kernel from the two
# rocprofv3 PMC passes (FETCH_SIZE, WRITE_SIZE, scaled by a 1 GiB copy) recorded
# in profiles/step_lambda_hbm_traffic_pmc.md.  They describe the kernel built
# from sources with this hash; once those change the figure is reported as null.
AT_TRAFFIC = {"src_sha16": "6698e33937ae40e8", "fetch_bytes": 0.000951e9, "write_bytes": 7.0313e9,
              "valu_instructions": 38170657092}  # SQ_INSTS_VALU (wave instructions) per launch
# single-issue FP32 vector rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_ISSUE_SPEC = 256 * 4 * 16 * 2.4e9
AT_SOURCES = ("smx_triplet.hip", "smx_device.h", "smx_maps.h")

N_EDM, D_EDM = 65536, 64
N_GRAM, D_GRAM = 32768, 512
N_AT = 8192
N_MAP4 = 1024  # 4-simplex map-only comparison: 8^4-element tiles, nb = 128
ALL_MAPS = ("lambda", "bbox", "linear", "recursive", "recursive_launch")
QUICK_MAPS = ("lambda", "bbox")
N_LIFE = 32768  # Life on the 2-simplex: 512 x 512 tiles of 64 x 64 cells, upper triangle
QUAD_RC = 2.0  # contact radius of the 4-point contact count (mean contact degree ~34)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-compare", action="store_true")
    p.add_argument("--quick-compare", action="store_true",
                   help="compare lambda with the bounding box only (no linear / recursive maps; map-only "
                        "parallel spaces of these two): a short run for tracing")
    p.add_argument("--only", default="", help="comma list of edm,gram,at (default all)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="first run one 1 GiB device-to-device copy (known traffic) to scale "
                        "rocprofv3 FETCH_SIZE / WRITE_SIZE readings")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(each step is one GPU's share at its real shape)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1610_07394_amd as smx
    import synth

    only = set(args.only.split(",")) if args.only else {"edm", "gram", "at"}
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating inputs")
    X2 = torch.from_numpy(synth.workload_input("edm_n65536_d64")).to(dev)
    X3 = torch.from_numpy(synth.workload_input("gram_n32768_d512")).to(dev)
    X5 = torch.from_numpy(synth.workload_input("at_lj_n8192")).to(dev)
    D2 = torch.empty(N_EDM * (N_EDM + 1) // 2, dtype=torch.float32, device=dev) if "edm" in only else None
    D3 = torch.empty(N_GRAM * (N_GRAM + 1) // 2, dtype=torch.float32, device=dev) if "gram" in only else None
    ws3 = torch.empty(smx.workspace_bytes(1, N_GRAM, D_GRAM, 2), dtype=torch.uint8, device=dev)
    ws5 = torch.empty(smx.workspace_bytes(2, N_AT), dtype=torch.uint8, device=dev)
    pot = smx.Pot(nu=1.0, at=True, lj=True, eps=1.0, sigma=1.0, rc=3.0)
    gradE = torch.ones(1, dtype=torch.float64, device=dev)
    dX = torch.empty((N_AT, 3), dtype=torch.float32, device=dev)

    def step(kind="lambda", parts=only):
        if "edm" in parts:
            smx.edm_packed(X2, kind, "fp32", out=D2)
        if "gram" in parts:
            smx.edm_packed(X3, kind, "split_bf16", out=D3, ws=ws3)
        if "at" in parts:
            # forward + backward: energy and dE/dx in one pass, then the
            # backward scaling by the incoming gradient
            E, G = smx.triplet_energy_grad(X5, pot, kind, ws=ws5)
            smx._check(smx.lib().smx_scale_grad(G.data_ptr(), N_AT, gradE.data_ptr(), dX.data_ptr(),
                                                smx._stream()))

    elements = {
        "edm": N_EDM * (N_EDM + 1) // 2,
        "gram": N_GRAM * (N_GRAM + 1) // 2,
        "at": math.comb(N_AT, 3) + math.comb(N_AT, 2),
    }
    total_elems = sum(elements[p] for p in only)

    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del src, dst
    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    smx.profile_enable(True)
    smx.profile_reset()
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    kern = {k: smx.profile_read(k) for k in smx.KERNELS}
    smx.profile_enable(False)
    kavg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kern.items()}
    value = total_elems / (ms_step / 1e3)

    # ---- per-component rooflines (algorithmic units per launch / avg launch time)
    comps = {}
    if "edm" in only:
        t = kavg["edm_diff"] / 1e3
        e = elements["edm"]
        comps["edm_fp32_n65536_d64"] = {
            "elements": e, "kernel_ms": kavg["edm_diff"], "elements_per_s": e / t,
            "alu_tflops": 3 * D_EDM * e / t / 1e12, "alu_frac": 3 * D_EDM * e / t / PEAK_FP32,
            "hbm_gbs": 4 * e / t / 1e9, "hbm_frac": 4 * e / t / PEAK_HBM}
    if "gram" in only:
        t = kavg["edm_gram"] / 1e3
        e = elements["gram"]
        comps["edm_split_bf16_n32768_d512"] = {
            "elements": e, "kernel_ms": kavg["edm_gram"], "prep_ms": kavg["gram_prep"],
            "elements_per_s": e / (t + kavg["gram_prep"] / 1e3),
            "mfma_tflops": 3 * 2 * D_GRAM * e / t / 1e12, "mfma_frac": 3 * 2 * D_GRAM * e / t / PEAK_BF16,
            "hbm_gbs": 4 * e / t / 1e9, "hbm_frac": 4 * e / t / PEAK_HBM}
    if "gram" in only:
        # the plain BF16 Gram form on the same input: bound by the 4-byte output stores
        smx.edm_packed(X3, "lambda", "bf16", out=D3, ws=ws3)
        torch.cuda.synchronize()
        smx.profile_enable(True)
        smx.profile_reset()
        for _ in range(args.steps):
            smx.edm_packed(X3, "lambda", "bf16", out=D3, ws=ws3)
        ms, c = smx.profile_read("edm_gram")
        smx.profile_enable(False)
        t = ms / c / 1e3
        e = elements["gram"]
        byts = 4 * e + 2 * N_GRAM * D_GRAM * 2  # packed FP32 output + the BF16 operand once
        # measured write ceilings on this GPU for the same 2.15 GB output: a plain
        # streaming fill of the buffer, and the packed-triangle tile stores of the
        # same kernel with 32 input dimensions (1/16 of the matrix-core work)
        fill = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        D3.fill_(0.0)
        fill[0].record()
        for _ in range(args.steps):
            D3.fill_(1.0)
        fill[1].record()
        torch.cuda.synchronize()
        t_fill = fill[0].elapsed_time(fill[1]) / args.steps / 1e3
        X3s = X3[:, :32].contiguous()
        smx.edm_packed(X3s, "lambda", "bf16", out=D3, ws=ws3)
        torch.cuda.synchronize()
        smx.profile_enable(True)
        smx.profile_reset()
        for _ in range(args.steps):
            smx.edm_packed(X3s, "lambda", "bf16", out=D3, ws=ws3)
        ms32, c32 = smx.profile_read("edm_gram")
        smx.profile_enable(False)
        del X3s
        # the tile-contiguous layout (one 64 KB run per 128 x 128 tile), plain and split
        log("tile-contiguous EDM layout")
        Dt = torch.empty(smx.edm_tiled_len(N_GRAM), dtype=torch.float32, device=dev)
        tiled = {}
        for prec in ("bf16", "split_bf16"):
            smx.edm_tiled(X3, "lambda", prec, out=Dt, ws=ws3)
            torch.cuda.synchronize()
            smx.profile_enable(True)
            smx.profile_reset()
            for _ in range(args.steps):
                smx.edm_tiled(X3, "lambda", prec, out=Dt, ws=ws3)
            mt, ct = smx.profile_read("edm_gram")
            smx.profile_enable(False)
            tt = mt / ct / 1e3
            bt = 4 * Dt.numel()
            tiled[prec] = {"kernel_ms": tt * 1e3, "elements_per_s": e / tt, "bytes_written": bt,
                           "hbm_gbs": bt / tt / 1e9, "hbm_frac": bt / tt / PEAK_HBM,
                           "mfma_frac": (3 if prec == "split_bf16" else 1) * 2 * D_GRAM * e / tt / PEAK_BF16}
        del Dt
        comps["edm_bf16_n32768_d512"] = {
            "elements": e, "kernel_ms": ms / c, "elements_per_s": e / t,
            "mfma_tflops": 2 * D_GRAM * e / t / 1e12, "mfma_frac": 2 * D_GRAM * e / t / PEAK_BF16,
            "hbm_gbs": byts / t / 1e9, "hbm_frac": byts / t / PEAK_HBM,
            "write_ceiling_fill_gbs": 4 * e / t_fill / 1e9,
            "write_ceiling_packed_d32_ms": ms32 / c32,
            "frac_of_packed_d32": (ms32 / c32) / (ms / c),
            "tiled_layout": tiled}
    if "at" in only:
        t = kavg["triplet_grad"] / 1e3
        tri = math.comb(N_AT, 3)
        comps["at_lj_n8192_fwd_bwd"] = {
            "triplets": tri, "pairs": math.comb(N_AT, 2), "kernel_ms": kavg["triplet_grad"],
            "lj_ms": kavg["lj"], "triplets_per_s": tri / t,
            "alu_tflops": AT_FLOPS_FWD_BWD * tri / t / 1e12, "alu_frac": AT_FLOPS_FWD_BWD * tri / t / PEAK_FP32}

    # the Axilrod-Teller workload at n = 2048 (forward + backward, one fused pass)
    # and the energy-only kernel at n = 2048 and n = 8192, beside the step
    if "at" in only:
        log("Axilrod-Teller n = 2048 forward + backward, energy-only kernels")
        X4 = torch.from_numpy(synth.workload_input("at_n2048")).to(dev)
        at_only = smx.Pot(nu=1.0, at=True, lj=False)
        ws4 = torch.empty(smx.workspace_bytes(2, X4.shape[0]), dtype=torch.uint8, device=dev)

        def timed(fn, kernel, reps):
            fn()
            torch.cuda.synchronize()
            smx.profile_enable(True)
            smx.profile_reset()
            for _ in range(reps):
                fn()
            ms, c = smx.profile_read(kernel)
            smx.profile_enable(False)
            return ms / c

        n4 = X4.shape[0]
        tri4 = math.comb(n4, 3)
        reps = max(args.steps, 10)
        t_fb = timed(lambda: smx.triplet_energy_grad(X4, at_only, "lambda", ws=ws4), "triplet_grad", reps)
        t_fb_bb = timed(lambda: smx.triplet_energy_grad(X4, at_only, "bbox", ws=ws4), "triplet_grad", reps)
        t_f = timed(lambda: smx.triplet_energy(X4, at_only, "lambda", ws=ws4), "triplet_energy", reps)
        t_f8 = timed(lambda: smx.triplet_energy(X5, at_only, "lambda", ws=ws5), "triplet_energy", args.steps)
        tri5 = math.comb(N_AT, 3)
        comps["at_n2048_fwd_bwd"] = {
            "triplets": tri4, "kernel_ms": t_fb, "bbox_kernel_ms": t_fb_bb, "speedup_lambda_vs_bbox": t_fb_bb / t_fb,
            "triplets_per_s": tri4 / (t_fb / 1e3),
            "alu_tflops": AT_FLOPS_FWD_BWD * tri4 / (t_fb / 1e3) / 1e12,
            "alu_frac": AT_FLOPS_FWD_BWD * tri4 / (t_fb / 1e3) / PEAK_FP32,
            "per_unit": "80 declared flops per triplet (20 forward + 60 backward), 1.4296e9 triplets per launch"}
        comps["at_n2048_fwd"] = {
            "triplets": tri4, "kernel_ms": t_f, "triplets_per_s": tri4 / (t_f / 1e3),
            "alu_tflops": AT_FLOPS_FWD * tri4 / (t_f / 1e3) / 1e12,
            "alu_frac": AT_FLOPS_FWD * tri4 / (t_f / 1e3) / PEAK_FP32,
            "per_unit": "20 declared flops per triplet (forward), 1.4296e9 triplets per launch"}
        comps["at_n8192_fwd"] = {
            "triplets": tri5, "kernel_ms": t_f8, "triplets_per_s": tri5 / (t_f8 / 1e3),
            "alu_tflops": AT_FLOPS_FWD * tri5 / (t_f8 / 1e3) / 1e12,
            "alu_frac": AT_FLOPS_FWD * tri5 / (t_f8 / 1e3) / PEAK_FP32,
            "per_unit": "20 declared flops per triplet (forward), 9.159e10 triplets per launch"}
        del ws4

    # packed per-triplet energies, n = 2048 (the write-bound 3-simplex workload;
    # measured beside the step, not part of it)
    if "at" in only and not args.no_compare:
        log("packed triplet energies, n = 2048")
        Xp = torch.from_numpy(synth.workload_input("at_n2048")).to(dev)
        npk = Xp.shape[0]
        mpk = npk * (npk - 1) * (npk - 2) // 6
        Ep = torch.empty(mpk, dtype=torch.float32, device=dev)
        pk = {}
        for kind in ("lambda", "bbox"):
            smx.triplet_packed(Xp, 1.0, kind, out=Ep)
            torch.cuda.synchronize()
            smx.profile_enable(True)
            smx.profile_reset()
            for _ in range(args.steps):
                smx.triplet_packed(Xp, 1.0, kind, out=Ep)
            ms, c = smx.profile_read("triplet_packed")
            smx.profile_enable(False)
            pk[kind] = ms / c
        ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev[0].record()
        for _ in range(args.steps):
            Ep.fill_(1.0)
        ev[1].record()
        torch.cuda.synchronize()
        t_fill = ev[0].elapsed_time(ev[1]) / args.steps / 1e3
        t = pk["lambda"] / 1e3
        # the same energies in the tile-contiguous layout (one 128 KB run per tile)
        del Ep
        mt = smx.triplet_tiled_len(npk)
        Et = torch.empty(mt, dtype=torch.float32, device=dev)
        smx.triplet_packed_tiled(Xp, 1.0, "lambda", out=Et)
        torch.cuda.synchronize()
        smx.profile_enable(True)
        smx.profile_reset()
        for _ in range(args.steps):
            smx.triplet_packed_tiled(Xp, 1.0, "lambda", out=Et)
        ms_t, c_t = smx.profile_read("triplet_tiled")
        smx.profile_enable(False)
        tt = ms_t / c_t / 1e3
        comps["at_packed_n2048"] = {
            "triplets": mpk, "kernel_ms": pk["lambda"], "bbox_ms": pk["bbox"], "triplets_per_s": mpk / t,
            "hbm_gbs": 4 * mpk / t / 1e9, "hbm_frac": 4 * mpk / t / PEAK_HBM,
            "write_ceiling_fill_gbs": 4 * mpk / t_fill / 1e9,
            "tiled_layout": {"kernel_ms": tt * 1e3, "triplets_per_s": mpk / tt, "bytes_written": 4 * mt,
                             "hbm_gbs": 4 * mt / tt / 1e9, "hbm_frac": 4 * mt / tt / PEAK_HBM},
            "per_unit": "4 bytes written per triplet (i < j < k), 1.430e9 triplets per launch; tiled layout: "
                        "4 bytes per slot of the 45760 tiles of 32^3"}
        del Et, Xp

    # 4-point contacts over the 4-simplex, n = 8192 (measured beside the step):
    # contact words over the 2-simplex, then the 4-cliques per 64^4 tile
    if "at" in only and not args.no_compare:
        log("4-point contacts, n = 8192")
        qd = {}
        ws4 = torch.empty(smx.workspace_bytes(3, N_AT), dtype=torch.uint8, device=dev)
        cnt = torch.empty(1, dtype=torch.int64, device=dev)
        for kind in QUICK_MAPS if args.quick_compare else ALL_MAPS:
            smx.quad_contacts(X5, QUAD_RC, kind, out=cnt, ws=ws4)
            torch.cuda.synchronize()
            smx.profile_enable(True)
            smx.profile_reset()
            for _ in range(args.steps):
                smx.quad_contacts(X5, QUAD_RC, kind, out=cnt, ws=ws4)
            w_ms, w_c = smx.profile_read("quad_words")
            q_ms, q_c = smx.profile_read("quad")
            smx.profile_enable(False)
            qd[kind] = {"words_ms": w_ms / w_c, "quad_ms": q_ms / q_c,
                        "blocks": smx.parallel_blocks(4, -(-N_AT // 64), 1, kind)}
        nq = math.comb(N_AT, 4)
        t = (qd["lambda"]["words_ms"] + qd["lambda"]["quad_ms"]) / 1e3
        comps["quad_contacts_n8192"] = {
            "quadruplets": nq, "contact_radius": QUAD_RC, "cliques": int(cnt.item()),
            "ms": t * 1e3, "quadruplets_per_s": nq / t, "maps": qd,
            "speedup_lambda_vs_bbox": (qd["bbox"]["words_ms"] + qd["bbox"]["quad_ms"]) / (t * 1e3),
            "per_unit": "64^4 quadruplets per tile (map decoded one id per lane, tiles counted one per wave at a time); 3 KB of contact words read per mapped tile"}
        del ws4

    # Life on the 2-simplex of cells, n = 32768, tile-contiguous 64 x 64 byte
    # tiles (measured beside the step): one generation per launch, buffers alternated
    if not args.no_compare:
        log(f"life on the 2-simplex, n = {N_LIFE}")
        ln = smx.life_len(N_LIFE)
        La = torch.from_numpy(synth.bits_flat(ln, seed=31, density=0.3)).to(dev)
        Lb = torch.empty_like(La)
        lf = {}
        for kind in QUICK_MAPS if args.quick_compare else ALL_MAPS:
            smx.simplex_life(La, N_LIFE, kind, out=Lb)
            torch.cuda.synchronize()
            smx.profile_enable(True)
            smx.profile_reset()
            for s_ in range(args.steps):
                src, dst = (La, Lb) if s_ % 2 == 0 else (Lb, La)
                smx.simplex_life(src, N_LIFE, kind, out=dst)
            ms, c = smx.profile_read("life")
            smx.profile_enable(False)
            lf[kind] = {"kernel_ms": ms / c, "blocks": smx.parallel_blocks(2, N_LIFE // 64, 1, kind)}
        cells = N_LIFE * (N_LIFE + 1) // 2
        t = lf["lambda"]["kernel_ms"] / 1e3
        comps["life_n32768"] = {
            "cells": cells, "ms": t * 1e3, "cells_per_s": cells / t, "hbm_gbs": 2 * ln / t / 1e9,
            "hbm_frac": 2 * ln / t / PEAK_HBM, "maps": lf,
            "speedup_lambda_vs_bbox": lf["bbox"]["kernel_ms"] / (t * 1e3),
            "per_unit": "8192 bytes per 64 x 64 tile (4096 read, 4096 written; the 260-cell ring from "
                        "neighbouring tiles not counted), 131328 tiles per launch"}
        del La, Lb

    # dominant kernel (largest time per step)
    per_step = {k: kern[k][0] / args.steps for k in kern}
    dom = max(per_step, key=per_step.get)
    if dom == "triplet_grad":
        t = kavg[dom] / 1e3
        ach = AT_FLOPS_FWD_BWD * math.comb(N_AT, 3) / t
        traffic = at_traffic()
        roof = {"kernel": "at_kernel<lambda, grad>", "bound": "alu", "achieved": ach / 1e12,
                "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": ach / PEAK_FP32,
                "traffic": None if traffic is None else traffic[0] + traffic[1],
                "traffic_fetch_bytes": None if traffic is None else traffic[0],
                "traffic_write_bytes": None if traffic is None else traffic[1],
                "per_unit": "80 flops per triplet (20 forward + 60 backward), 9.159e10 triplets per launch",
                "frac_basis": "declared flops against the packed-FP32 vector peak; the kernel is built without "
                              "packed FP32, so its physical ceiling is the VALU issue rate (valu_issue)"}
        if traffic is not None:
            issue = traffic[2] * 64 / t  # VALU lane-instructions per second
            ceil = valu_ceiling(smx, torch, dev)
            roof["valu_issue"] = {"lane_instructions_per_s": issue, "per_triplet": traffic[2] * 64 / math.comb(N_AT, 3),
                                  "spec_single_issue": VALU_ISSUE_SPEC, "frac_spec": issue / VALU_ISSUE_SPEC,
                                  "measured_fma_chain": ceil, "frac_measured": issue / ceil}
    elif dom == "edm_diff":
        t = kavg[dom] / 1e3
        ach = 3 * D_EDM * elements["edm"] / t
        roof = {"kernel": "edm_diff_kernel<lambda>", "bound": "alu", "achieved": ach / 1e12,
                "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s", "frac": ach / PEAK_FP32, "traffic": None,
                "per_unit": "3 d flops per pair, 2.1475e9 pairs per launch"}
    else:
        t = kavg[dom] / 1e3
        ach = 3 * 2 * D_GRAM * elements["gram"] / t
        roof = {"kernel": "edm_gram_kernel<lambda, split>", "bound": "mfma", "achieved": ach / 1e12,
                "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s", "frac": ach / PEAK_BF16, "traffic": None,
                "per_unit": "6 d flops per pair (3 BF16 products), 5.369e8 pairs per launch"}

    # ---- lambda vs bounding box vs linear (same steps, timed after the main loop)
    compare = None
    if not args.no_compare:
        compare = {}
        log("step on the other maps")
        for kind in (QUICK_MAPS if args.quick_compare else ALL_MAPS)[1:]:
            step(kind)  # warm
            torch.cuda.synchronize()
            smx.profile_enable(True)
            smx.profile_reset()
            for _ in range(args.steps):
                step(kind)
            kk = {k: smx.profile_read(k) for k in ("edm_diff", "edm_gram", "triplet_grad", "lj")}
            smx.profile_enable(False)
            compare[kind] = {k: (v[0] / v[1] if v[1] else None) for k, v in kk.items()}
        compare["lambda"] = {k: kavg[k] for k in ("edm_diff", "edm_gram", "triplet_grad", "lj")}
        for base in ("bbox",) if args.quick_compare else ("bbox", "recursive", "recursive_launch"):
            sp = {}
            for k in ("edm_diff", "edm_gram", "triplet_grad"):
                if compare[base].get(k) and compare["lambda"].get(k):
                    sp[k] = compare[base][k] / compare["lambda"][k]
            compare[f"speedup_lambda_vs_{base}"] = sp
        # map-only parallel spaces (paper-like granularity: rho = 16 pairs, rho = 8 triplets)
        # "visit" = every element of every mapped tile is touched (count + id
        # checksum); "count" = each mapped block adds its tile's closed-form
        # count, so the time is the map plus the launched blocks alone.
        mo = {}
        log("map-only parallel spaces")
        for kind in QUICK_MAPS if args.quick_compare else ("lambda", "bbox", "linear", "lambda_below", "recursive",
                                                          "recursive_launch"):
            for m, n, rho in ((2, N_EDM, 16), (3, N_AT, 8), (4, N_MAP4, 8)):
                if m == 4 and kind == "lambda_below":
                    continue  # not defined for the 4-simplex
                visit = {2: smx.simplex_map2, 3: smx.simplex_map3, 4: smx.simplex_map4}[m]
                runs = (("visit", lambda: visit(n, rho, kind, strict=(m >= 3), tiles=False)),
                        ("count", lambda: smx.simplex_count(m, n, rho, kind, strict=(m >= 3))))
                for what, fn in runs:
                    fn()
                    torch.cuda.synchronize()
                    smx.profile_enable(True)
                    smx.profile_reset()
                    for _ in range(3):
                        fn()
                    ms, c = smx.profile_read(f"map{m}")
                    smx.profile_enable(False)
                    mo[f"{what}{m}_{kind}_n{n}_rho{rho}_ms"] = ms / c
                # the map alone, one lane per logical block id (no block per tile)
                nb = n // rho
                smx.simplex_decode(m, nb, kind)
                torch.cuda.synchronize()
                smx.profile_enable(True)
                smx.profile_reset()
                for _ in range(3):
                    smx.simplex_decode(m, nb, kind)
                ms, c = smx.profile_read("decode")
                smx.profile_enable(False)
                mo[f"decode{m}_{kind}_nb{nb}_ms"] = ms / c
        compare["map_only"] = mo

    # ---- CPU baseline: the FP64 oracle on a bounded sample, host cores
    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle)")
        cpu = cpu_baseline(only, elements, total_elems)
        log("measured errors against the oracle")
        accuracy = measured_errors(only, smx, torch, dev, X2, X3, X5, D2, D3, ws3, ws5, pot)
        for name, key in (("edm_fp32_n65536_d64", "edm_fp32_n65536_d64"),
                          ("edm_split_bf16_n32768_d512", "gram_split_bf16_n32768_d512"),
                          ("edm_bf16_n32768_d512", "gram_bf16_n32768_d512"),
                          ("at_lj_n8192_fwd_bwd", "at_lj_n8192"), ("at_n2048_fwd_bwd", "at_n2048")):
            if name in comps and key in accuracy:
                comps[name]["max_err"] = accuracy[key]

    out = {
        "metric": "simplex elements/sec (lambda map) for packed EDM + AT/LJ fwd+bwd",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded: N(0,1) EDM inputs, RSA particles in a cube of side 20, dmin 0.8)",
        "config": {
            "workload": "step = edm_fp32 n=65536 d=64 + edm_gram split-bf16 n=32768 d=512 + "
                        "axilrod-teller + lennard-jones fwd+bwd n=8192 (lambda maps)",
            "elements_per_step": total_elems,
            "parts": sorted(only),
        },
        "roofline": roof,
        "components": comps,
        "kernel_ms_avg": kavg,
        "compare": compare,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
    }
    print(json.dumps(out))


def at_traffic():
    """(fetch, write) HBM bytes per AT gradient launch, or None if the kernel
    sources changed since the counters were taken."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1610_07394_amd", "csrc")
    h = hashlib.sha256()
    for f in AT_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != AT_TRAFFIC["src_sha16"]:
        return None
    return AT_TRAFFIC["fetch_bytes"], AT_TRAFFIC["write_bytes"], AT_TRAFFIC["valu_instructions"]


def valu_ceiling(smx, torch, dev):
    """Measured FP32 VALU issue rate (lane operations / s): the library's FMA-chain
    probe, best of three launches timed with events on the current stream."""
    blocks, iters = 8192, 2048
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    best = None
    for _ in range(4):
        ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev[0].record()
        smx._check(smx.lib().smx_probe_valu(out.data_ptr(), blocks, iters, smx._stream()))
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        best = ms if best is None else min(best, ms)
    return blocks * 256 * iters * 64 / (best / 1e3)


def measured_errors(only, smx, torch, dev, X2, X3, X5, D2, D3, ws3, ws5, pot):
    """Errors of the GPU results against the FP64 oracle on bounded samples
    (the same metrics as the parity tests): packed EDM rows 0..R of each
    workload, every precision of the Gram input; Axilrod-Teller + LJ energies
    and gradient rows at n = 8192, the whole energy and gradient at n = 2048."""
    import json

    import numpy as np

    import oracle
    import synth

    out = {}
    refs = {}

    def edm_err(Xn, Dg, rows, scale_form):
        n = Xn.shape[0]
        if (n, rows) not in refs:
            refs[(n, rows)] = oracle.edm_rows(Xn, 0, rows)
        ref = refs[(n, rows)]
        got = Dg[:ref.shape[0]].cpu().numpy().astype(np.float64)
        ii = np.repeat(np.arange(rows), n - np.arange(rows))
        jj = np.concatenate([np.arange(i, n) for i in range(rows)])
        diag = ii == jj
        off = ~diag
        res = {"pairs": int(ref.shape[0]), "rows": f"0..{rows}", "diagonal_exact_zero": bool((got[diag] == 0).all())}
        rel = np.abs(got[off] - ref[off]) / ref[off]
        res["max_rel_err"] = float(rel.max())
        res["mean_rel_err"] = float(rel.mean())
        if scale_form:
            nrm = (Xn.astype(np.float64) ** 2).sum(1)
            sc = np.abs(got[off] - ref[off]) / (nrm[ii[off]] + nrm[jj[off]])
            res["max_err_vs_norms"] = float(sc.max())
            res["metric"] = "|D^ - D| / (|x_i|^2 + |x_j|^2), off the diagonal (max_rel_err: |D^ - D| / D)"
            res["value"] = res["max_err_vs_norms"]
        else:
            res["metric"] = "|D^ - D| / D, off the diagonal"
            res["value"] = res["max_rel_err"]
        return res

    if "edm" in only:
        smx.edm_packed(X2, "lambda", "fp32", out=D2)
        torch.cuda.synchronize()
        out["edm_fp32_n65536_d64"] = edm_err(synth.workload_input("edm_n65536_d64"), D2, 1024, False)
    if "gram" in only:
        Xg = synth.workload_input("gram_n32768_d512")
        for prec, key in (("bf16", "gram_bf16_n32768_d512"), ("split_bf16", "gram_split_bf16_n32768_d512"),
                          ("fp32", "gram_input_fp32_diff_n32768_d512")):
            smx.edm_packed(X3, "lambda", prec, out=D3, ws=ws3)
            torch.cuda.synchronize()
            out[key] = edm_err(Xg, D3, 1024, True)
    if "at" in only:
        X = synth.workload_input("at_lj_n8192")
        E, G = smx.triplet_energy_grad(X5, pot, "lambda", ws=ws5)
        torch.cuda.synchronize()
        E = E.cpu().numpy()
        G = G.cpu().numpy().astype(np.float64)
        rows = list(range(0, N_AT, 256))
        g_ref = oracle.at_grad_rows(X, rows, 1.0) + oracle.lj_grad(X, 1.0, 1.0, 3.0)[rows]
        lj_ref = oracle.lj_energy(X, 1.0, 1.0, 3.0)
        res = {"metric": "max_i |G^_i - G_i| / max_i |G_i| over the sampled rows (forces = -G)",
               "gradient_rows": len(rows),
               "value": float(np.linalg.norm(G[rows] - g_ref, axis=1).max() / np.linalg.norm(g_ref, axis=1).max()),
               "lj_energy_rel_err": abs(E[2] - lj_ref) / abs(lj_ref)}
        gold = os.path.join(ROOT, "tests", "golden", "expected.json")
        if os.path.exists(gold):  # the full AT energy, stored by the oracle-only golden script
            e_at = json.load(open(gold))["at_lj_n8192"]["at_energy"]
            res["at_energy_rel_err"] = abs(E[1] - e_at) / abs(e_at)
        out["at_lj_n8192"] = res
        X4n = synth.workload_input("at_n2048")
        X4 = torch.from_numpy(X4n).to(dev)
        at_only = smx.Pot(nu=1.0, at=True, lj=False)
        E4, G4 = smx.triplet_energy_grad(X4, at_only, "lambda")
        torch.cuda.synchronize()
        e_ref = oracle.at_energy(X4n, 1.0)
        g4_ref = oracle.at_grad(X4n, 1.0)
        G4 = G4.cpu().numpy().astype(np.float64)
        out["at_n2048"] = {"metric": "max_i |G^_i - G_i| / max_i |G_i| over all 2048 rows (forces = -G)",
                           "value": float(np.linalg.norm(G4 - g4_ref, axis=1).max() / np.linalg.norm(g4_ref, axis=1).max()),
                           "energy_rel_err": abs(float(E4[0].item()) - e_ref) / abs(e_ref)}
    return out


def cpu_baseline(only, elements, total_elems):
    import numpy as np

    import oracle
    import synth

    cores = oracle.threads()
    secs_per_step = 0.0
    samples = []
    if "edm" in only:
        X = synth.workload_input("edm_n65536_d64")
        r = 16384
        t0 = time.perf_counter()
        oracle.edm_rows(X, 0, r)
        dt = time.perf_counter() - t0
        e = oracle.packed_offset(r, N_EDM)
        secs_per_step += elements["edm"] * dt / e
        samples.append(f"EDM d=64 rows 0..{r} ({e} pairs, {dt:.2f}s)")
    if "gram" in only:
        X = synth.workload_input("gram_n32768_d512")
        r = 4096
        t0 = time.perf_counter()
        oracle.edm_rows(X, 0, r)
        dt = time.perf_counter() - t0
        e = oracle.packed_offset(r, N_GRAM)
        secs_per_step += elements["gram"] * dt / e
        samples.append(f"EDM d=512 rows 0..{r} ({e} pairs, {dt:.2f}s)")
    if "at" in only:
        X = synth.workload_input("at_lj_n8192")
        i1 = 240
        t0 = time.perf_counter()
        oracle.at_energy(X, 1.0, 0, i1)
        dt_e = time.perf_counter() - t0
        tri_e = sum(math.comb(N_AT - 1 - i, 2) for i in range(i1))
        rows = list(range(0, 8192, 256))
        t0 = time.perf_counter()
        oracle.at_grad_rows(X, rows, 1.0)
        dt_g = time.perf_counter() - t0
        tri_g = len(rows) * math.comb(N_AT - 1, 2)
        t0 = time.perf_counter()
        oracle.lj_energy(X)
        oracle.lj_grad(X)
        dt_lj = time.perf_counter() - t0
        tri = math.comb(N_AT, 3)
        secs_per_step += tri * dt_e / tri_e + tri * dt_g / tri_g + dt_lj
        samples.append(f"AT energy i<{i1} ({tri_e} triplets, {dt_e:.2f}s); AT gradient of {len(rows)} particles "
                       f"({tri_g} triplets, {dt_g:.2f}s); LJ energy+gradient full ({dt_lj:.2f}s)")
    # one core, for reference: the FP32-input EDM rows and the AT energy on small samples
    single = {}
    oracle.set_threads(1)
    try:
        if "edm" in only:
            X = synth.workload_input("edm_n65536_d64")
            t0 = time.perf_counter()
            oracle.edm_rows(X, 0, 512)
            single["edm_pairs_per_s"] = oracle.packed_offset(512, N_EDM) / (time.perf_counter() - t0)
        if "at" in only:
            X = synth.workload_input("at_lj_n8192")
            t0 = time.perf_counter()
            oracle.at_energy(X, 1.0, 0, 4)
            single["at_energy_triplets_per_s"] = (sum(math.comb(N_AT - 1 - i, 2) for i in range(4))
                                                  / (time.perf_counter() - t0))
    finally:
        oracle.set_threads(cores)
    return {"value": total_elems / secs_per_step, "unit": "elements/s", "cores": cores, "kind": "oracle",
            "sample": "; ".join(samples) + " -- scaled to one full step", "single_core": single}


if __name__ == "__main__":
    main()
