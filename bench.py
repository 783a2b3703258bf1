"""Throughput benchmark: visibility x component evaluations per second.

Workload: the MWA-like predict (128 tiles = 8128 baselines, 14 times at 8 s,
32 channels of 80 kHz at 182 MHz; 20000 points, 2000 Gaussians, 2 shapelets
with n1 + n2 <= 54; Gaussian primary beam), synthetic and seeded.  A step is
one vp_predict of the whole sky into resident complex64 visibilities on the
mixed-precision path; the FP64 path is timed beside it.  Shapelets count as
their (N+1)(N+2)/2 basis functions.

The JSON line carries:
  roofline     -- the point/Gaussian tile kernel (the dominant kernel here),
                  vector-ALU bound: algorithmic VALU issue slots per launch /
                  its mean duration (HIP events on the launch stream) against
                  the chip's VALU issue peak;
  cpu_baseline -- the FP64 oracle on a bounded sample of rows, on the host's
                  cores, which also checks the GPU output on those rows;
  shapelet_contraction -- the shapelet kernel alone on the Fornax-like
                  workload (two lobes, n1 + n2 <= 70), per contraction mode:
                  algorithmic contraction FLOP/s (2 p_tot per visibility and
                  shapelet) against the FP32 MFMA peak, and the MFMA work the
                  kernel issues against the peak of the instruction type used; beside
                  them the FP64 vector-ALU path and its lookup-table variant of the
                  basis (the paper's simulator's evaluation), timed and checked the
                  same way.
                  `--only-shapelets` runs this leg alone (for profiling);
  truncation_sweep -- the paper's model truncation (Sec. 5.3) on its peel
                  observation: GPU time and error against the full model per
                  fraction of components kept;
  paper_peel   -- the paper's own peel at its scale: the p_max = 86 lobes on
                  its 46.8 M-visibility observation, predict + calibrate (10
                  iterations per time and channel) + subtract, timed, with
                  sampled cells checked against the oracle;
  calibrated_peel -- the large peel observation (256 tiles, 1 time, 384
                  channels, complex64 data holding the 10 N=80 shapelet
                  sources, each under its own synthetic tile gains, plus
                  noise): the sources peeled one after another with
                  calibration (Sec. 5.1) on the mixed path; time per source
                  split into prediction and gain solve, and the residual RMS
                  against plain (uncalibrated) subtraction;
  large_peel   -- the same observation with N(0, 1 Jy) data: the 10 sources
                  subtracted one after another (vp_subtract) and the whole sky
                  predicted, on the mixed path (complex64) and the FP64 path
                  (complex128), with RMS(R_gpu - R_ref) beside RMS(R_ref) on
                  sampled rows;
  serving      -- the serving stream: p50/p99 latency, throughput, the
                  persistent kernels' resident time against the same jobs
                  run back to back, and 8 requests checked against the
                  oracle; serving_full_hbm_budget repeats it with the
                  budget at 90% of free device memory.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic VALU issue slots per evaluation.  Every VALU instruction of a wave
# of 64 takes one 4-cycle issue slot of its SIMD; v_sin/v_cos/v_exp take one slot
# too and then run in the transcendental unit beside the vector ALU (measured: the
# kernel's VALU instructions, transcendentals included, fill 0.99 of the SIMD
# cycles at 4 cycles each, so they do not hold the issue port longer).
# With uniformly spaced channels (this workload) the mixed kernel evaluates the
# phasor of 3 channels of each 8 and the channel step, and rotates the others:
#   per 8 channels: 4 x (phase scale 1 + reduction 1 + convert 1 + sin 1 + cos 1)
#                   + 5 complex rotations x 4 + 8 complex MACs x 2 = 56
#   point:    56 / 8                                                       = 7
#   Gaussian: point + exponent scale 1 + exp2 1 + flux x envelope 1        = 10
#   per (row, component): u l + v m + w (n - 1), 3 FMAs shared by the row's channels
SLOTS_POINT, SLOTS_GAUSS, SLOTS_ROW_COMP = 7, 10, 3

# HBM bytes per launch of the point/Gaussian kernel on this workload, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a 1 GiB copy (summary in
# profiles/k_pg_tile_mwa-like_hbm-traffic.md), valid for the kernel source
# whose hash is recorded; reported as null once that source changes.
PG_TRAFFIC = {"bytes": 128.0e6 + 29.1e6, "source_sha256_16": "ce22dd23a7358942"}


# dense MFMA peaks and the FP64 vector peak (TFLOP/s)
MFMA_PEAK_F32 = 157.3
MFMA_PEAK_BF16 = 2500.0
VALU_PEAK_F64 = 78.6


def _shp_mfma_flops(nmax, n_vis, mode):
    """MFMA flops the shapelet kernel issues per launch: per 32 visibilities and
    32 x 32 coefficient block, K steps of 4 orders on v_mfma_f32_32x32x2f32
    (2 per step, 4096 flops each; only steps inside the triangle), or 2 parities
    x 6 (BF16 x3) or 3 (BF16 x2) v_mfma_f32_32x32x16_bf16 (32768 flops each)."""
    total = 0.0
    for N in nmax:
        q = N // 32
        for ch in range(q + 1):
            for mb in range(q - ch + 1):
                if mode == "f32":
                    total += 2 * min(8, (N - 32 * (ch + mb)) // 4 + 1) * 4096
                else:
                    total += 2 * (6 if mode == "bf16x3" else 3) * 32768
    return total * n_vis / 32.0


def shapelet_contraction(reps=5):
    """Shapelet kernel on the Fornax-like workload, per precision path: time per
    launch (HIP events on the launch stream), contraction FLOP/s and, against the
    oracle over every visibility of the workload, the maximum error relative to
    the total flux (complex128 output, so that the figure is the path's own)."""
    import torch

    import oracle
    import synth
    from paper_2005_09316_amd import vp

    obs, sky = synth.make_config(2)
    ctx = vp.vp_create_ctx(0, 0)
    oh, sh = vp.vp_create_obs(ctx, obs), vp.vp_create_sky(ctx, sky)
    nrows, K = obs.n_time * obs.n_bl, obs.n_chan
    out = torch.empty((nrows, K), dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    ptot = sum((int(n) + 1) * (int(n) + 2) // 2 for n in sky.s_nmax)
    alg_flops = 2.0 * ptot * obs.n_vis
    t0 = time.time()
    ref = oracle.predict(obs, sky).reshape(nrows, K)
    _log("fornax-like oracle over all %d visibilities: %.1f s on %d threads"
         % (obs.n_vis, time.time() - t0, oracle.max_threads()))
    res = {"workload": synth.CONFIG_NAMES[2], "n_vis": obs.n_vis, "nmax": [int(n) for n in sky.s_nmax],
           "algorithmic_flops_per_launch": alg_flops, "error": "max over all visibilities vs the oracle, "
           "relative to the channel's total flux", "modes": {}}
    for name, prec, mode, peak in (("mixed_bf16x3", vp.VP_PREC_MIXED, "bf16x3", MFMA_PEAK_BF16),
                                   ("mixed_bf16x2", vp.VP_PREC_MIXED_BF16X2, "bf16x2", MFMA_PEAK_BF16),
                                   ("fp32_only", vp.VP_PREC_FP32, "f32", MFMA_PEAK_F32),
                                   ("fp64_valu", vp.VP_PREC_FP64, None, VALU_PEAK_F64),
                                   ("lut_valu", vp.VP_PREC_LUT, None, VALU_PEAK_F64)):
        vp.vp_predict(ctx, sh, oh, prec, vp.VP_C128, out.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        vp.vp_profile(ctx, True)
        vp.vp_profile_read(ctx)
        for _ in range(reps):
            vp.vp_predict(ctx, sh, oh, prec, vp.VP_C128, out.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        c, t = vp.vp_profile_read(ctx)
        vp.vp_profile(ctx, False)
        ms = float(t[2] / max(c[2], 1))
        err = oracle.error_metric(out.cpu().numpy(), ref, obs, sky)
        r = {"kernel_ms": round(ms, 4),
             "algorithmic_tflops": round(alg_flops / ms / 1e9, 2),
             "frac_of_fp32_mfma_peak": round(alg_flops / ms / 1e9 / MFMA_PEAK_F32, 4),
             "own_peak_tflops": peak,
             "max_err_vs_oracle": err,
             "gate": {"mixed_bf16x3": 1e-6, "fp64_valu": 1e-11}.get(name)}
        if mode is not None:
            issued = _shp_mfma_flops(sky.s_nmax, obs.n_vis, mode)
            r["issued_mfma_tflops"] = round(issued / ms / 1e9, 2)
            r["issued_frac_of_own_peak"] = round(issued / ms / 1e9 / peak, 4)
        else:
            # vector-ALU paths: FP64 contraction against the FP64 vector peak
            r["frac_of_own_peak"] = round(alg_flops / ms / 1e9 / peak, 4)
        res["modes"][name] = r
        _log("shapelet kernel %s: %.3f ms, %.1f TFLOP/s algorithmic (%.1f%% of FP32 MFMA peak), "
             "max err %.2e" % (name, ms, r["algorithmic_tflops"], 100 * r["frac_of_fp32_mfma_peak"], err))
    vp.vp_destroy_sky(sh)
    vp.vp_destroy_obs(oh)
    vp.vp_destroy_ctx(ctx)
    del out
    torch.cuda.empty_cache()
    return res


def truncation_sweep(check_rows=8, fracs=(1.0, 0.95, 0.9, 0.8, 0.7, 0.5), orders=(86, 78, 70, 63, 54, 40)):
    """The paper's compute-vs-accuracy lever (Sec. 5.3): truncate the MS CLEAN-
    like model and the two p_max = 86 shapelet lobes by cumulative absolute
    flux (and the lobes by order), predict the peel observation on the mixed
    path, and report the GPU time beside the error of the truncated model
    against the oracle's full model on sampled rows (relative to the full
    model's total flux)."""
    import torch

    import oracle
    import synth
    from paper_2005_09316_amd import truncate, vp

    obs, clean, lobes = synth.make_paper_cost_comparison()
    ctx = vp.vp_create_ctx(0, 0)
    oh = vp.vp_create_obs(ctx, obs)
    nrows = obs.n_time * obs.n_bl
    out = torch.empty((nrows, obs.n_chan), dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    rows = np.sort(np.random.default_rng(7).choice(nrows, check_rows, replace=False))
    res = {"n_vis": obs.n_vis, "check_rows": check_rows, "models": {}}

    def eff_order(sky):
        m = 0
        for s in range(sky.n_shp):
            N = int(sky.s_nmax[s])
            c = sky.coeffs[int(sky.s_coeff_off[s]):int(sky.s_coeff_off[s]) + (N + 1) * (N + 2) // 2]
            n1, n2 = truncate._orders(N)
            nz = np.flatnonzero(c)
            m = max(m, int((n1[nz] + n2[nz]).max()) if nz.size else 0)
        return m

    for name, sky in (("clean", clean), ("shapelet", lobes)):
        ref = oracle.predict(obs, sky, rows=rows)
        variants = [("flux", f) + tuple(truncate.truncate_by_flux(sky, f)) for f in fracs]
        if name == "shapelet":
            for n in orders:
                t = truncate.truncate_by_order(sky, n)
                full_flux = truncate.component_flux(sky)[0]
                kept_flux = truncate.component_flux(t)[0]
                variants.append(("order", n, t, int(np.count_nonzero(kept_flux)), full_flux.size,
                                 float(kept_flux.sum() / full_flux.sum())))
        rows_out = []
        for rule, param, t, n, ntot, frac in variants:
            sh = vp.vp_create_sky(ctx, t)
            vp.vp_predict(ctx, sh, oh, vp.VP_PREC_MIXED, vp.VP_C128, out.data_ptr(), stream.cuda_stream)
            torch.cuda.synchronize()
            vp.vp_profile(ctx, True)
            vp.vp_profile_read(ctx)
            reps = 2
            t0 = time.perf_counter()
            for _ in range(reps):
                vp.vp_predict(ctx, sh, oh, vp.VP_PREC_MIXED, vp.VP_C128, out.data_ptr(), stream.cuda_stream)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) * 1e3 / reps
            c, tk = vp.vp_profile_read(ctx)
            vp.vp_profile(ctx, False)
            got = out[torch.as_tensor(rows, device="cuda")].cpu().numpy()
            err = oracle.error_metric(got, ref, obs, sky)
            vp.vp_destroy_sky(sh)
            r = {"rule": rule, "param": param, "kept": int(n), "of": int(ntot),
                 "kept_frac": round(n / ntot, 4), "flux_frac": round(frac, 5),
                 "gpu_ms": round(wall, 3),
                 "kernel_ms": round(float((tk[1] + tk[2]) / max(c[1], 1)), 3),
                 "err_vs_full_model": err}
            if name == "shapelet":
                r["effective_order"] = eff_order(t)
            rows_out.append(r)
            _log("truncation %s %s=%s: kept %d/%d (%.0f%%, %.1f%% of |flux|), %.2f ms, error %.2e"
                 % (name, rule, param, n, ntot, 100.0 * n / ntot, 100.0 * frac, wall, err))
        res["models"][name] = rows_out
    vp.vp_destroy_obs(oh)
    vp.vp_destroy_ctx(ctx)
    del out
    torch.cuda.empty_cache()
    return res


def calibrated_peel(n_iter=10, check_chan=(17,)):
    """Workload 4's observation: data = sum over the 10 shapelet sources of
    g_i g_j^* V_s (a gain table of its own per source) + N(0, 1 Jy) noise,
    complex64, resident.  Timed: the 10 vp_peel calls in sequence (predict
    into the workspace, solve gains per (time, channel), subtract).  Beside
    it: the same data after plain vp_subtract of the 10 sources, and a check
    of the last source's gains on one channel against the oracle."""
    import torch

    import oracle
    import synth
    from paper_2005_09316_amd import vp

    obs, sky = synth.make_config(4)
    n_ant = int(obs.n_tiles)
    a1, a2 = synth.antenna_pairs(n_ant)
    srcs = [synth.select_components(sky, points=[], gauss=[], shapelets=[k]) for k in range(sky.n_shp)]
    ctx = vp.vp_create_ctx(0, 0)
    oh = vp.vp_create_obs(ctx, obs)
    handles = [vp.vp_create_sky(ctx, s) for s in srcs]
    stream = torch.cuda.current_stream()
    shape = (obs.n_time, obs.n_bl, obs.n_chan)
    rng = np.random.default_rng(4040)
    gains_true = [synth.random_gains(rng, obs.n_time, obs.n_chan, n_ant) for _ in srcs]
    # build the data on the device: sum_s g_ant1 g_ant2^* V_s + noise
    data0 = torch.from_numpy(synth.noise_c64(shape, seed=4041)).to("cuda")
    tmp = torch.empty(shape, dtype=torch.complex64, device="cuda")
    i1 = torch.as_tensor(a1, dtype=torch.long, device="cuda")
    i2 = torch.as_tensor(a2, dtype=torch.long, device="cuda")
    for h, G in zip(handles, gains_true):
        vp.vp_predict(ctx, h, oh, vp.VP_PREC_MIXED, vp.VP_C64, tmp.data_ptr(), stream.cuda_stream)
        g = torch.from_numpy(G).to(torch.complex64).to("cuda")          # [T, K, n_ant]
        corr = (g[:, :, i1] * torch.conj(g[:, :, i2])).permute(0, 2, 1)  # [T, B, K]
        data0 += corr * tmp
    torch.cuda.synchronize()
    rms0 = float(torch.sqrt(torch.mean(torch.abs(data0) ** 2)))
    # plain subtraction for comparison
    d = data0.clone()
    for h in handles:
        vp.vp_subtract(ctx, h, oh, vp.VP_PREC_MIXED, vp.VP_C64, d.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    rms_plain = float(torch.sqrt(torch.mean(torch.abs(d) ** 2)))
    gains = torch.empty((len(handles), obs.n_time, obs.n_chan, n_ant), dtype=torch.complex128, device="cuda")

    def run():
        for s, h in enumerate(handles):
            vp.vp_peel(ctx, h, oh, a1, a2, n_ant, n_iter, vp.VP_PREC_MIXED, vp.VP_C64, d.data_ptr(),
                       gains[s].data_ptr(), stream.cuda_stream)

    d.copy_(data0)
    run()  # warm: tables and workspace
    torch.cuda.synchronize()
    d.copy_(data0)
    torch.cuda.synchronize()
    vp.vp_profile(ctx, True)
    vp.vp_profile_read(ctx)
    t0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    c, tk = vp.vp_profile_read(ctx)
    vp.vp_profile(ctx, False)
    rms_peel = float(torch.sqrt(torch.mean(torch.abs(d) ** 2)))
    rms_noise = math.sqrt(2.0)
    # check: the first source peeled from the original data, on sampled
    # channels, against the oracle's solution from the same data
    ks = np.asarray(check_chan)
    sub = dataclasses.replace(obs, n_chan=int(ks.size), freq_hz=obs.freq_hz[ks])
    d1 = data0.clone()
    g1 = torch.empty((obs.n_time, obs.n_chan, n_ant), dtype=torch.complex128, device="cuda")
    vp.vp_peel(ctx, handles[0], oh, a1, a2, n_ant, n_iter, vp.VP_PREC_MIXED, vp.VP_C64, d1.data_ptr(),
               g1.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    M = oracle.predict(sub, srcs[0]).reshape(obs.n_time, obs.n_bl, ks.size)
    din = data0[:, :, torch.as_tensor(ks, device="cuda")].cpu().numpy().astype(np.complex128)
    g_ref, r_ref = oracle.peel(din, M, a1, a2, n_ant, n_iter)
    gg = g1[:, torch.as_tensor(ks, device="cuda"), :].cpu().numpy()
    p = gg[:, :, a1] * np.conj(gg[:, :, a2])
    p_ref = g_ref[:, :, a1] * np.conj(g_ref[:, :, a2])
    r_got = d1[:, :, torch.as_tensor(ks, device="cuda")].cpu().numpy().astype(np.complex128)
    check = {"source": 0, "channels": ks.tolist(),
             "gain_products_rel_err": float(np.abs(p - p_ref).max() / np.abs(p_ref).max()),
             "residual_err_vs_total_flux": oracle.error_metric(r_got, r_ref, sub, srcs[0])}
    res = {"n_vis": obs.n_vis, "n_sources": len(handles), "n_ant": n_ant, "n_iter": n_iter,
           "cells": obs.n_time * obs.n_chan, "ms_total": round(wall, 3),
           "ms_per_source": round(wall / len(handles), 3),
           "predict_kernel_ms": round(float(tk[1] + tk[2]), 3),
           "gain_solve_kernel_ms": round(float(tk[3]), 3), "gain_solve_launches": int(c[3]),
           "rms_data_jy": rms0, "rms_after_plain_subtract_jy": rms_plain,
           "rms_after_calibrated_peel_jy": rms_peel, "rms_noise_jy": rms_noise,
           "oracle_check": check}
    _log("calibrated peel: %d sources x %.2f ms (predict %.2f ms, gain solve %.2f ms in total); rms %.3f -> plain "
         "%.3f, peeled %.3f (noise %.3f) Jy; check %s" % (len(handles), wall / len(handles), tk[1] + tk[2], tk[3],
                                                         rms0, rms_plain, rms_peel, rms_noise, check))
    for h in handles:
        vp.vp_destroy_sky(h)
    vp.vp_destroy_obs(oh)
    vp.vp_destroy_ctx(ctx)
    del d, d1, data0, tmp, gains, g1
    torch.cuda.empty_cache()
    return res


def paper_peel(n_iter=10, check=((14, 383), (0, 0), (7, 191))):
    """The paper's peel (Sec. 5.1) at its own scale: the two p_max = 86
    shapelet lobes on the peel observation (128 tiles, 15 x 8 s, 384 x 80 kHz
    = 46.8 M visibilities), data = the lobes under synthetic tile gains (one
    set per time and channel) + N(0, 1 Jy) noise, complex64.  Timed: one
    vp_peel with 10 Gauss-Newton iterations per (time, channel) cell (5760
    cells; the cell tables take three launches), i.e. predict + calibrate +
    subtract.  Checked: gains and residual of a few cells against the
    oracle (its own model and lstsq steps on the same data)."""
    import torch

    import oracle
    import synth
    from paper_2005_09316_amd import vp

    obs, _clean, lobes = synth.make_paper_cost_comparison()
    n_ant = int(obs.n_tiles)
    a1, a2 = synth.antenna_pairs(n_ant)
    ctx = vp.vp_create_ctx(0, 0)
    oh, sh = vp.vp_create_obs(ctx, obs), vp.vp_create_sky(ctx, lobes)
    shape = (obs.n_time, obs.n_bl, obs.n_chan)
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(5050)
    G = synth.random_gains(rng, obs.n_time, obs.n_chan, n_ant)
    data0 = torch.from_numpy(synth.noise_c64(shape, seed=5051)).to("cuda")
    tmp = torch.empty(shape, dtype=torch.complex64, device="cuda")
    vp.vp_predict(ctx, sh, oh, vp.VP_PREC_MIXED, vp.VP_C64, tmp.data_ptr(), stream.cuda_stream)
    g = torch.from_numpy(G).to(torch.complex64).to("cuda")
    i1 = torch.as_tensor(a1, dtype=torch.long, device="cuda")
    i2 = torch.as_tensor(a2, dtype=torch.long, device="cuda")
    data0 += (g[:, :, i1] * torch.conj(g[:, :, i2])).permute(0, 2, 1) * tmp
    del tmp
    torch.cuda.synchronize()
    rms0 = float(torch.sqrt(torch.mean(torch.abs(data0) ** 2)))
    d = data0.clone()
    gains = torch.empty((obs.n_time, obs.n_chan, n_ant), dtype=torch.complex128, device="cuda")
    vp.vp_peel(ctx, sh, oh, a1, a2, n_ant, n_iter, vp.VP_PREC_MIXED, vp.VP_C64, d.data_ptr(), gains.data_ptr(),
               stream.cuda_stream)  # warm: tables, workspace
    torch.cuda.synchronize()
    d.copy_(data0)
    torch.cuda.synchronize()
    vp.vp_profile(ctx, True)
    vp.vp_profile_read(ctx)
    t0 = time.perf_counter()
    vp.vp_peel(ctx, sh, oh, a1, a2, n_ant, n_iter, vp.VP_PREC_MIXED, vp.VP_C64, d.data_ptr(), gains.data_ptr(),
               stream.cuda_stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    c, tk = vp.vp_profile_read(ctx)
    vp.vp_profile(ctx, False)
    rms1 = float(torch.sqrt(torch.mean(torch.abs(d) ** 2)))
    checks = []
    for (t, k) in check:
        sub = dataclasses.replace(obs, n_time=1, uvw_m=np.ascontiguousarray(obs.uvw_m[t:t + 1]),
                                  n_chan=1, freq_hz=obs.freq_hz[k:k + 1])
        M = oracle.predict(sub, lobes).reshape(-1)
        v = data0[t, :, k].cpu().numpy().astype(np.complex128)
        g_ref = oracle.calibrate_cell(v, M, a1, a2, n_ant, n_iter)
        r_ref = v - g_ref[a1] * np.conj(g_ref[a2]) * M
        gg = gains[t, k].cpu().numpy()
        p, p_ref = gg[a1] * np.conj(gg[a2]), g_ref[a1] * np.conj(g_ref[a2])
        r = d[t, :, k].cpu().numpy().astype(np.complex128)
        F = float(oracle.total_flux(sub, lobes)[0])
        checks.append({"time": t, "channel": k,
                       "gain_products_rel_err": float(np.abs(p - p_ref).max() / np.abs(p_ref).max()),
                       "residual_err_vs_total_flux": float(np.abs(r - r_ref).max() / F)})
    res = {"n_vis": obs.n_vis, "n_ant": n_ant, "cells": obs.n_time * obs.n_chan, "n_iter": n_iter,
           "source": "2 shapelet lobes, p_max = 86 (7656 basis functions)",
           "ms_total": round(wall, 3), "predict_kernel_ms": round(float(tk[1] + tk[2]), 3),
           "calibration_ms": round(float(tk[3]), 3), "calibration_launches": int(c[3]),
           "rms_data_jy": rms0, "rms_residual_jy": rms1, "rms_noise_jy": math.sqrt(2.0),
           "oracle_checks": checks}
    _log("paper peel: %.1f ms (predict %.1f ms, calibration %.1f ms in %d launches); rms %.2f -> %.3f Jy "
         "(noise %.3f); checks %s" % (wall, tk[1] + tk[2], tk[3], c[3], rms0, rms1, math.sqrt(2.0), checks))
    vp.vp_destroy_sky(sh)
    vp.vp_destroy_obs(oh)
    vp.vp_destroy_ctx(ctx)
    del d, data0, gains
    torch.cuda.empty_cache()
    return res


def large_peel(check_rows=64, full_rows=4, reps=3):
    """Workload 4 (12.5M visibilities): the 10 bright shapelets subtracted one
    after another from resident N(0, 1 Jy) data, on the mixed path (complex64)
    and the FP64 path (complex128), and the whole sky (100000 points, 5000
    Gaussians, 10 shapelets) predicted on both.  The residual R = D - sum_k
    V_k is checked on sampled rows against the oracle's: RMS(R_gpu - R_ref)
    beside RMS(R_ref), and the error relative to the peeled flux; the full-sky
    prediction likewise on fewer rows (the oracle's cost)."""
    import torch

    import oracle
    import synth
    from paper_2005_09316_amd import vp

    obs, sky = synth.make_config(4)
    nrows, K = obs.n_time * obs.n_bl, obs.n_chan
    rng = np.random.default_rng(4400)
    rows = np.sort(rng.choice(nrows, check_rows, replace=False))
    frows = rows[:full_rows]
    data = synth.noise_c64((nrows, K), seed=4401)
    shp_sky = synth.select_components(sky, points=[], gauss=[], shapelets=None)
    t0 = time.perf_counter()
    r_ref = data[rows].astype(np.complex128) - oracle.predict(obs, shp_sky, rows=rows)
    v_full_ref = oracle.predict(obs, sky, rows=frows)
    t_oracle = time.perf_counter() - t0
    ctx = vp.vp_create_ctx(0, 0)
    oh = vp.vp_create_obs(ctx, obs)
    peel = [vp.vp_create_sky(ctx, synth.select_components(sky, points=[], gauss=[], shapelets=[k]))
            for k in range(sky.n_shp)]
    full = vp.vp_create_sky(ctx, sky)
    stream = torch.cuda.current_stream()
    rsel = torch.as_tensor(rows, device="cuda")
    res = {"n_vis": obs.n_vis, "n_sources": sky.n_shp, "check_rows": int(rows.size), "full_sky_check_rows": int(frows.size),
           "oracle_s": round(t_oracle, 2)}
    for name, prec, dtype, tdt in (("mixed", vp.VP_PREC_MIXED, vp.VP_C64, torch.complex64),
                                   ("fp64", vp.VP_PREC_FP64, vp.VP_C128, torch.complex128)):
        d0 = torch.from_numpy(data).to("cuda").to(tdt)
        d = d0.clone()

        def subtract_all():
            for h in peel:
                vp.vp_subtract(ctx, h, oh, prec, dtype, d.data_ptr(), stream.cuda_stream)

        subtract_all()  # warm: tables
        ms_sub = []
        for _ in range(reps):
            d.copy_(d0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            subtract_all()
            e1.record(stream)
            torch.cuda.synchronize()
            ms_sub.append(e0.elapsed_time(e1))
        got = d[rsel].cpu().numpy().astype(np.complex128)
        diff = got - r_ref
        out = torch.empty((nrows, K), dtype=tdt, device="cuda")
        vp.vp_predict(ctx, full, oh, prec, dtype, out.data_ptr(), stream.cuda_stream)  # warm
        ms_full = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            vp.vp_predict(ctx, full, oh, prec, dtype, out.data_ptr(), stream.cuda_stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms_full.append(e0.elapsed_time(e1))
        vf = out[torch.as_tensor(frows, device="cuda")].cpu().numpy().astype(np.complex128)
        res[name] = {
            "output": "complex64" if dtype == vp.VP_C64 else "complex128",
            "ms_10_subtractions": round(min(ms_sub), 3),
            "rms_residual_diff_jy": float(np.sqrt(np.mean(np.abs(diff) ** 2))),
            "rms_residual_ref_jy": float(np.sqrt(np.mean(np.abs(r_ref) ** 2))),
            "residual_err_vs_peeled_flux": oracle.error_metric(got, r_ref, obs, shp_sky),
            "ms_full_sky_predict": round(min(ms_full), 3),
            "full_sky_evals_per_s": obs.n_vis * sky.nominal_components() / (min(ms_full) * 1e-3),
            "full_sky_err_vs_total_flux": oracle.error_metric(vf, v_full_ref, obs, sky),
        }
        _log("large peel (%s): 10 subtractions %.2f ms, rms(R_gpu - R_ref) %.3e Jy of rms(R_ref) %.3f Jy, "
             "error / peeled flux %.2e; full sky %.2f ms (%.3e evals/s), error / total flux %.2e"
             % (name, res[name]["ms_10_subtractions"], res[name]["rms_residual_diff_jy"],
                res[name]["rms_residual_ref_jy"], res[name]["residual_err_vs_peeled_flux"],
                res[name]["ms_full_sky_predict"], res[name]["full_sky_evals_per_s"],
                res[name]["full_sky_err_vs_total_flux"]))
        del d0, d, out
        torch.cuda.empty_cache()
    for h in peel + [full]:
        vp.vp_destroy_sky(h)
    vp.vp_destroy_obs(oh)
    vp.vp_destroy_ctx(ctx)
    return res


def _pg_source_hash():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2005_09316_amd", "csrc", "vp_kernels.hip")).read()
    a, b = src.index("// point + Gaussian tile kernel"), src.index("// shapelet tile on MFMA")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _host_info():
    """Host CPU as the oracle runs on it: logical CPUs, model name, OpenMP threads."""
    import oracle
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "omp_threads": oracle.max_threads()}


def cpu_plan(c1_rate, c1_sample):
    """The oracle's rates on the host beside the GPU figures: one thread (a
    per-core rate) on the tiny workload and on a fixed subset of the MWA-like
    rows; all threads on the tiny workload, on the MWA-like sample (timed in
    the main leg), on every visibility of the Fornax-like workload, on a
    deterministic subset of the large peel's rows (extrapolated to the whole
    observation and labelled so), and on sampled rows of 8 serving requests."""
    import oracle
    import synth

    def timed(obs, sky, rows=None, nthreads=0):
        t0 = time.perf_counter()
        oracle.predict(obs, sky, rows=rows, nthreads=nthreads)
        dt = time.perf_counter() - t0
        nrow = len(rows) if rows is not None else obs.n_time * obs.n_bl
        ev = nrow * obs.n_chan * sky.nominal_components()
        return {"evals": ev, "s": round(dt, 3), "evals_per_s": ev / dt}

    host = _host_info()
    out = {"host": host, "one_thread": {}, "all_threads": {}}
    obs, sky = synth.make_config(0)
    out["one_thread"]["tiny"] = timed(obs, sky, nthreads=1)
    out["all_threads"]["tiny"] = timed(obs, sky)
    obs, sky = synth.make_config(1)
    rows = np.arange(0, obs.n_time * obs.n_bl, 1777)[:64]
    r = timed(obs, sky, rows=rows, nthreads=1)
    r["sample"] = "64 of %d (time, baseline) rows, every 1777th" % (obs.n_time * obs.n_bl)
    out["one_thread"]["mwa_like_subset"] = r
    out["all_threads"]["mwa_like_sample"] = {"evals_per_s": c1_rate, "sample": c1_sample}
    obs, sky = synth.make_config(2)
    r = timed(obs, sky)
    r["sample"] = "every visibility (%d)" % obs.n_vis
    out["all_threads"]["fornax_like_full"] = r
    obs, sky = synth.make_config(4)
    nrows = obs.n_time * obs.n_bl
    rows = np.arange(0, nrows, nrows // 16)[:16]
    r = timed(obs, sky, rows=rows)
    r["sample"] = "16 of %d baselines (every %dth), all 384 channels and all components" % (nrows, nrows // 16)
    r["extrapolated_full_s"] = round(r["s"] * nrows / len(rows), 1)
    r["extrapolated"] = True
    out["all_threads"]["large_peel_subset"] = r
    reqs = synth.make_requests(8)
    ev, dt = 0, 0.0
    for q in reqs:
        nr = q.obs.n_time * q.obs.n_bl
        rr = np.arange(0, nr, max(1, nr // 16))[:16]
        x = timed(q.obs, q.sky, rows=rr)
        ev += x["evals"]
        dt += x["s"]
    out["all_threads"]["serving_8_requests"] = {"evals": ev, "s": round(dt, 3), "evals_per_s": ev / dt,
                                                "sample": "16 rows of each of the first 8 stream requests"}
    _log("cpu plan: %s" % json.dumps(out))
    return out


def serve_stream(n_requests, rate_hz, budget_bytes):
    """Serving stream: Poisson arrivals of uneven predict / peel-subtract
    requests (tiles 64/128/256, 8-384 channels, 1-14 times, ~2000 points,
    ~200 Gaussians, 0-4 shapelets of order 20-80), submitted at their arrival
    times into one context with an HBM admission budget.  Sky models,
    observations and visibility buffers are resident before the stream
    starts; subtract requests run on complex64 data (device-drawn noise).
    Latency = completion - scheduled arrival."""
    import torch

    import synth
    from paper_2005_09316_amd import vp

    t0 = time.time()
    reqs = synth.make_requests(n_requests, rate_hz)
    ctx = vp.vp_create_ctx(0, budget_bytes)
    prepared = []
    for r in reqs:
        oh, sh = vp.vp_create_obs(ctx, r.obs), vp.vp_create_sky(ctx, r.sky)
        shape = (r.obs.n_time, r.obs.n_bl, r.obs.n_chan)
        if r.kind == "subtract":
            g = torch.Generator(device="cuda").manual_seed(r.noise_seed)
            buf = torch.randn(shape, dtype=torch.complex64, device="cuda", generator=g)
        else:
            buf = torch.empty(shape, dtype=torch.complex64, device="cuda")
        prepared.append((r, oh, sh, buf))
    torch.cuda.synchronize()
    _log("serving: %d requests prepared in %.1f s (%.1f GB of resident visibilities)"
         % (len(reqs), time.time() - t0, sum(p[3].numel() * 8 for p in prepared) / 1e9))
    start = time.monotonic_ns()
    pending = {}
    lat, done_t, evals = [], [], 0
    nxt = 0
    while nxt < len(prepared) or pending:
        now = time.monotonic_ns()
        while nxt < len(prepared) and start + int(prepared[nxt][0].t_arrival_s * 1e9) <= now:
            r, oh, sh, buf = prepared[nxt]
            arr = start + int(r.t_arrival_s * 1e9)
            kind = vp.VP_JOB_SUBTRACT if r.kind == "subtract" else vp.VP_JOB_PREDICT
            t = vp.vp_submit(ctx, kind, sh, oh, vp.VP_PREC_MIXED, vp.VP_C64, buf.data_ptr(), arr)
            pending[t] = (r, arr)
            nxt += 1
        for t in list(pending):
            res = vp.vp_poll(ctx, t)
            if res is not None:
                r, arr = pending.pop(t)
                if res["status"] != vp.VP_OK:
                    raise RuntimeError("serving job failed with %d" % res["status"])
                lat.append((res["t_done"] - arr) / 1e6)
                done_t.append(res["t_done"])
                evals += r.obs.n_vis * r.sky.nominal_components()
        time.sleep(0.0002)
    wall = (max(done_t) - start) / 1e9
    time.sleep(0.05)  # the persistent kernels' idle exit, so that their last launch is counted
    launches, resident_ms = vp.vp_serve_stats(ctx)
    # 8 requests spread over the stream against the oracle, on 16 sampled rows
    # each (a subtract request's data are the same seeded device noise again)
    import oracle
    check_errs = []
    for i in np.linspace(0, len(prepared) - 1, 8).astype(int):
        r, oh, sh, buf = prepared[i]
        nrows = r.obs.n_time * r.obs.n_bl
        rows = np.sort(np.random.default_rng(7000 + int(i)).choice(nrows, min(16, nrows), replace=False))
        sel = torch.as_tensor(rows, device="cuda")
        got = buf.reshape(nrows, r.obs.n_chan)[sel].cpu().numpy().astype(np.complex128)
        ref = oracle.predict(r.obs, r.sky, rows=rows)
        if r.kind == "subtract":
            g = torch.Generator(device="cuda").manual_seed(r.noise_seed)
            d0 = torch.randn(buf.shape, dtype=torch.complex64, device="cuda", generator=g)
            ref = d0.reshape(nrows, r.obs.n_chan)[sel].cpu().numpy().astype(np.complex128) - ref
            del d0
        check_errs.append(oracle.error_metric(got, ref, r.obs, r.sky) if r.sky.nominal_components() else 0.0)
    _log("serving: 8 requests against the oracle on 16 rows each, max error / total flux %.2e"
         % max(check_errs))
    # the same requests back to back through vp_predict / vp_subtract, for the
    # serving efficiency
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r, oh, sh, buf in prepared:
        fn = vp.vp_subtract if r.kind == "subtract" else vp.vp_predict
        fn(ctx, sh, oh, vp.VP_PREC_MIXED, vp.VP_C64, buf.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    standalone = time.perf_counter() - t0
    for r, oh, sh, buf in prepared:
        vp.vp_destroy_sky(sh)
        vp.vp_destroy_obs(oh)
    vp.vp_destroy_ctx(ctx)
    lat = np.asarray(lat)
    out = {"requests": len(reqs), "rate_hz": rate_hz, "budget_bytes": budget_bytes,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "max_ms": float(lat.max()), "wall_s": wall, "requests_per_s": len(reqs) / wall,
           "evals_per_s": evals / wall, "precision": "mixed", "output": "complex64",
           "back_to_back_evals_per_s": evals / standalone, "back_to_back_s": standalone,
           "kernel_launches": launches, "kernel_resident_s": resident_ms / 1e3,
           "resident_over_back_to_back": resident_ms / 1e3 / standalone,
           "oracle_check": {"requests": 8, "rows_each": 16, "max_err_vs_oracle": max(check_errs),
                            "gate": 1e-6}}
    _log("serving: p50 %.1f ms, p99 %.1f ms, %.2e evals/s over %.1f s; persistent kernel %d launches, "
         "resident %.2f s against %.2f s back to back" % (out["p50_ms"], out["p99_ms"], out["evals_per_s"], wall,
                                                       launches, resident_ms / 1e3, standalone))
    return out


def paper_cost_comparison():
    """The paper's Sec. 5.3 comparison on this chip: time to predict the peel
    observation from the MS CLEAN-like model (4540 points + 1791 Gaussians)
    and from the two p_max = 86 shapelet lobes (7656 basis functions), on the
    mixed and FP64 paths.  The paper found the shapelet model more than twice
    as expensive on its GPU simulator."""
    import torch

    import synth
    from paper_2005_09316_amd import vp

    obs, clean, lobes = synth.make_paper_cost_comparison()
    ctx = vp.vp_create_ctx(0, 0)
    oh = vp.vp_create_obs(ctx, obs)
    out = torch.empty((obs.n_time, obs.n_bl, obs.n_chan), dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    res = {"n_vis": obs.n_vis, "clean_components": clean.n_point + clean.n_gauss,
           "shapelet_basis_functions": lobes.n_basis()}
    for name, sky in (("clean", clean), ("shapelet", lobes)):
        sh = vp.vp_create_sky(ctx, sky)
        for pname, prec in (("mixed", vp.VP_PREC_MIXED), ("fp64", vp.VP_PREC_FP64)):
            vp.vp_predict(ctx, sh, oh, prec, vp.VP_C128, out.data_ptr(), stream.cuda_stream)
            torch.cuda.synchronize()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                vp.vp_predict(ctx, sh, oh, prec, vp.VP_C128, out.data_ptr(), stream.cuda_stream)
            torch.cuda.synchronize()
            res["%s_%s_ms" % (name, pname)] = (time.perf_counter() - t0) * 1e3 / reps
        vp.vp_destroy_sky(sh)
    for pname in ("mixed", "fp64"):
        res["shapelet_over_clean_%s" % pname] = res["shapelet_%s_ms" % pname] / res["clean_%s_ms" % pname]
    # what the paper states for the same comparison, on its hardware (Sec. 5.3)
    res["paper"] = {"shapelet_over_clean": "> 2", "hardware": "NVIDIA GeForce GTX 1080 Ti (12 GB)",
                    "simulator": "the authors' CUDA simulator", "absolute_times": "not stated"}
    vp.vp_destroy_obs(oh)
    vp.vp_destroy_ctx(ctx)
    _log("paper cost comparison: %s" % json.dumps(res))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--cpu-rows", type=int, default=12288)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cpu-plan", action="store_true", help="only the MWA-like oracle sample")
    ap.add_argument("--only-cpu-plan", action="store_true", help="run the oracle's host-rate plan alone")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-budget-gb", type=float, default=4.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-paper-cost", action="store_true")
    ap.add_argument("--no-shapelets", action="store_true", help="skip the shapelet-contraction leg")
    ap.add_argument("--no-truncation", action="store_true", help="skip the truncation sweep")
    ap.add_argument("--no-peel", action="store_true", help="skip the calibrated-peel leg")
    ap.add_argument("--only-peel", action="store_true", help="run the calibrated-peel leg alone")
    ap.add_argument("--no-paper-peel", action="store_true", help="skip the paper-scale calibrated peel")
    ap.add_argument("--no-large-peel", action="store_true", help="skip the large-peel subtraction leg")
    ap.add_argument("--only-large-peel", action="store_true", help="run the large-peel subtraction leg alone")
    ap.add_argument("--only-paper-peel", action="store_true", help="run the paper-scale calibrated peel alone")
    ap.add_argument("--only-shapelets", action="store_true",
                    help="run only the shapelet-contraction leg and print its JSON")
    ap.add_argument("--only-serve", action="store_true", help="run the serving stream alone and print its JSON")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device-to-device copy first (its HBM counters scale the kernels')")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2005_09316_amd import vp

    if args.only_shapelets:
        print(json.dumps(shapelet_contraction()), flush=True)
        return
    if args.only_peel:
        print(json.dumps(calibrated_peel()), flush=True)
        return
    if args.only_cpu_plan:
        print(json.dumps(cpu_plan(None, None)), flush=True)
        return
    if args.only_large_peel:
        print(json.dumps(large_peel()), flush=True)
        return
    if args.only_paper_peel:
        print(json.dumps(paper_peel()), flush=True)
        return
    if args.only_serve:
        print(json.dumps(serve_stream(args.serve_requests, args.serve_rate, int(args.serve_budget_gb * 1e9))),
              flush=True)
        return

    t_gen = time.time()
    obs, sky = synth.make_config(1)
    _log("workload generated in %.1f s: %d vis, %d points, %d gaussians, %d shapelets (%d basis)"
         % (time.time() - t_gen, obs.n_vis, sky.n_point, sky.n_gauss, sky.n_shp, sky.n_basis()))
    n_vis = obs.n_vis
    nominal = n_vis * sky.nominal_components()
    nrows, K = obs.n_time * obs.n_bl, obs.n_chan

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        _log("copy calibration: 1 GiB read + 1 GiB written")

    ctx = vp.vp_create_ctx(0, 0)
    oh, sh = vp.vp_create_obs(ctx, obs), vp.vp_create_sky(ctx, sky)
    stream = torch.cuda.current_stream()
    out = torch.empty((obs.n_time, obs.n_bl, obs.n_chan), dtype=torch.complex64, device="cuda")

    def step(prec, buf, dtype):
        vp.vp_predict(ctx, sh, oh, prec, dtype, buf.data_ptr(), stream.cuda_stream)

    # ---- mixed path (the measured value) ----
    for _ in range(args.warmup):
        step(vp.VP_PREC_MIXED, out, vp.VP_C64)
    torch.cuda.synchronize()
    vp.vp_profile(ctx, True)
    vp.vp_profile_read(ctx)  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(vp.VP_PREC_MIXED, out, vp.VP_C64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    counts, tot_ms = vp.vp_profile_read(ctx)
    vp.vp_profile(ctx, False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = nominal / (ms_step * 1e-3)
    pg_ms = tot_ms[1] / max(counts[1], 1)
    shp_ms = tot_ms[2] / max(counts[2], 1)
    _log("mixed: %.3f ms/step, %.3e evals/s; pg kernel %.3f ms, shapelet kernel %.3f ms"
         % (ms_step, value, pg_ms, shp_ms))

    # ---- FP64 path, for the speedup ----
    out64 = torch.empty((obs.n_time, obs.n_bl, obs.n_chan), dtype=torch.complex128, device="cuda")
    ms64, value64 = float("nan"), float("nan")
    if args.fp64_steps > 0:
        step(vp.VP_PREC_FP64, out64, vp.VP_C128)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.fp64_steps):
            step(vp.VP_PREC_FP64, out64, vp.VP_C128)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) * 1e3 / args.fp64_steps
        value64 = nominal / (ms64 * 1e-3)
        _log("fp64: %.3f ms/step, %.3e evals/s" % (ms64, value64))

    # ---- roofline of the point/Gaussian kernel ----
    pg_evals_pt = nrows * K * sky.n_point
    pg_evals_g = nrows * K * sky.n_gauss
    slots = (pg_evals_pt * SLOTS_POINT + pg_evals_g * SLOTS_GAUSS
             + nrows * (sky.n_point + sky.n_gauss) * SLOTS_ROW_COMP)
    achieved = slots / (pg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_pg_tile<mixed, uniform channels>", "achieved": round(achieved, 3),
                "peak": round(VALU_PEAK_TOPS, 3), "unit": "Tops/s (VALU issue slots)",
                "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": PG_TRAFFIC["bytes"] if _pg_source_hash() == PG_TRAFFIC["source_sha256_16"] else None,
                "traffic_unit": "bytes per launch (HBM read + write)",
                "kernel_ms": round(pg_ms, 4), "shapelet_kernel_ms": round(shp_ms, 4)}

    # ---- sampled parity + CPU baseline (oracle) ----
    cpu = None
    err = None
    if not args.no_cpu:
        import oracle
        rng = np.random.default_rng(5)
        rows = np.sort(rng.choice(nrows, args.cpu_rows, replace=False))
        got = out.reshape(nrows, K)[torch.as_tensor(rows, device="cuda")].cpu().numpy()
        threads = oracle.max_threads()
        t0 = time.perf_counter()
        ref = oracle.predict(obs, sky, rows=rows, nthreads=threads)
        dt = time.perf_counter() - t0
        err = oracle.error_metric(got, ref, obs, sky)
        sample_evals = len(rows) * K * sky.nominal_components()
        cpu = {"value": sample_evals / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": "%d of %d (time, baseline) rows x all %d channels x all components; %.1f s"
                         % (len(rows), nrows, K, dt)}
        _log("oracle: %.3e evals/s on %d threads; sampled error / total flux = %.3e" % (cpu["value"], threads, err))
        cpu["gpu_over_oracle"] = value / cpu["value"]
        if not args.no_cpu_plan:
            cpu["plan"] = cpu_plan(cpu["value"], cpu["sample"])

    vp.vp_destroy_sky(sh)
    vp.vp_destroy_obs(oh)
    vp.vp_destroy_ctx(ctx)
    del out, out64
    torch.cuda.empty_cache()

    paper_cost = None if args.no_paper_cost else paper_cost_comparison()
    shp = None if args.no_shapelets else shapelet_contraction()
    trunc = None if args.no_truncation else truncation_sweep()
    peel = None if args.no_peel else calibrated_peel()
    ppeel = None if args.no_paper_peel else paper_peel()
    lpeel = None if args.no_large_peel else large_peel()

    serving = serving_full = None
    if not args.no_serve:
        serving = serve_stream(args.serve_requests, args.serve_rate, int(args.serve_budget_gb * 1e9))
        # the same stream once more with the full-HBM budget (0: 90% of free device memory)
        serving_full = serve_stream(args.serve_requests, args.serve_rate, 0)

    line = {
        "metric": "vis x component evals/s (mixed precision, err <= 1e-6 vs FP64 oracle); p50/p99 latency",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (f64 phase)", "data": "synthetic",
        "config": {"workload": synth.CONFIG_NAMES[1], "n_vis": n_vis,
                   "components": {"point": sky.n_point, "gaussian": sky.n_gauss, "shapelet": sky.n_shp,
                                  "shapelet_basis": sky.n_basis()},
                   "nominal_evals_per_step": nominal, "precision": "mixed", "output": "complex64",
                   "fp64_path": {"evals_per_s": value64, "ms_per_step": ms64},
                   "speedup_vs_fp64": value / value64,
                   "evals_per_s_shapelet_as_one": n_vis * (sky.n_point + sky.n_gauss + sky.n_shp) / (ms_step * 1e-3),
                   "sampled_err_vs_oracle": err},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
        "serving_full_hbm_budget": serving_full,
        "paper_cost_comparison": paper_cost,
        "shapelet_contraction": shp,
        "truncation_sweep": trunc,
        "calibrated_peel": peel,
        "paper_peel": ppeel,
        "large_peel": lpeel,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
