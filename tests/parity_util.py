"""Helpers for the GPU-vs-oracle parity tests."""
import numpy as np

import oracle

# Parity bars (GPU vs FP64 oracle, stamps where both report CONVERGED):
# |dx|, |dy| <= 1e-3 px, |de| <= 1e-4, relative 1e-3 on Re and n.
BAR_X = 1e-3
BAR_E = 1e-4
BAR_REL = 1e-3


def run_gpu(shape, batch, opts=None, device="cuda:0"):
    import torch
    db = shape.DeviceBatch.from_host(batch, device)
    out = shape.pipeline(db, opts, want_perr=True)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def oracle_opts_like(gpu_opts, **kw):
    """Oracle options with the same stage rules as the GPU run; the fit keeps
    the oracle's own tight tolerance unless overridden."""
    o = oracle.opts(max_iter_centroid=gpu_opts.max_iter_centroid,
                    max_iter_moments=gpu_opts.max_iter_moments,
                    k_gain=gpu_opts.k_gain, tol_x=gpu_opts.tol_x, tol_g=gpu_opts.tol_g,
                    gmax=gpu_opts.gmax, lambda0=gpu_opts.lambda0, chi2_rtol=gpu_opts.chi2_rtol,
                    n0=gpu_opts.n0, moffat_beta=gpu_opts.moffat_beta,
                    free_mask=gpu_opts.free_mask, linear_init=gpu_opts.linear_init)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def compare(gpu, ref, free_mask=0xFF, label=""):
    """Return a dict of parity statistics (GPU vs oracle)."""
    st_g, st_o = gpu["status"].astype(np.uint32), ref["status"]
    conv = lambda st, k: (st[:, k] & oracle.CONVERGED) != 0
    out = {}
    # centroid stage: starting estimates and centre
    cg, co = gpu["centroid"], ref
    # a centre that left the stamp (LOST) follows diverging dynamics; compare the rest
    lost = ((st_g[:, 0] | st_o[:, 0]) & (oracle.LOST | oracle.BAD_INPUT | oracle.NONFINITE_INPUT)) != 0
    ok0 = np.isfinite(cg[:, 0]) & ~lost
    out["n"] = len(st_g)
    out["centroid_dxy"] = float(np.abs(cg[ok0, :2] - co["xy"][ok0]).max()) if ok0.any() else 0.0
    out["r50_rel"] = float(np.abs(cg[ok0, 5] / co["mom"][ok0, 5] - 1).max()) if ok0.any() else 0.0
    out["sigw_rel"] = float(np.abs(cg[ok0, 4] / co["mom"][ok0, 4] - 1).max()) if ok0.any() else 0.0
    out["status0_agree"] = float((st_g[:, 0] == st_o[:, 0]).mean())
    # moments stage
    both1 = conv(st_g, 1) & conv(st_o, 1)
    mg, mo = gpu["moments"], ref["mom"]
    out["moments_both"] = int(both1.sum())
    out["moments_dxy"] = float(np.abs(mg[both1, :2] - mo[both1, :2]).max()) if both1.any() else 0.0
    out["moments_de"] = float(np.abs(mg[both1, 2:4] - mo[both1, 2:4]).max()) if both1.any() else 0.0
    # the fit's starting size (record slot 8 on the GPU, slot 6 of the oracle's)
    fg, fo = np.isfinite(mg[both1, 8]), np.isfinite(mo[both1, 6])
    out["size_defined_agree"] = float((fg == fo).mean()) if both1.any() else 1.0
    fin = fg & fo
    out["size_rel"] = float(np.abs(mg[both1, 8][fin] / mo[both1, 6][fin] - 1).max()) if fin.any() else 0.0
    out["status1_agree"] = float((st_g[:, 1] == st_o[:, 1]).mean())
    # fit
    both2 = conv(st_g, 2) & conv(st_o, 2)
    pg, po = gpu["p"], ref["p"]
    out["fit_gpu_conv"] = int(conv(st_g, 2).sum())
    out["fit_oracle_conv"] = int(conv(st_o, 2).sum())
    out["fit_both"] = int(both2.sum())
    if both2.any():
        d = np.abs(pg[both2] - po[both2])
        rel = np.abs(pg[both2] / po[both2] - 1)
        out["fit_dxy"] = float(d[:, :2].max())
        out["fit_de"] = float(d[:, 2:4].max())
        out["fit_re_rel"] = float(rel[:, 4].max())
        out["fit_n_rel"] = float(rel[:, 5].max())
        out["fit_i0_rel"] = float(rel[:, 6].max())
        out["fit_sky_rel"] = float(rel[:, 7].max())
        out["fit_x_ok"] = float((d[:, :2].max(1) <= BAR_X).mean())
        out["fit_e_ok"] = float((d[:, 2:4].max(1) <= BAR_E).mean())
        out["fit_rel_ok"] = float((rel[:, 4:6].max(1) <= BAR_REL).mean())
        worst = np.argsort(-rel[:, 4:6].max(1))[:3]
        out["worst_idx"] = [int(i) for i in np.flatnonzero(both2)[worst]]
    print(label, {k: (round(v, 7) if isinstance(v, float) else v) for k, v in out.items()})
    return out
