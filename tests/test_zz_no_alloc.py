"""GPU: shape_fit_queue_static, the work-queue fit on the library's static
workspace (no allocation), against the queue calls with a caller-owned
workspace on the same stamps: two calls in a row, the second on a smaller
batch, each bit-identical to the workspace form."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_static_queue_fit_matches_workspace_queue():
    import torch

    import paper_1203_0571_amd as shape
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cases = (("uneven", 3000, dict(team=2, team_min_side=64)),   # Sersic + Moffat, any side
             ("sersic64h", 1024, dict(team=1)))                   # FP16, one side
    for workload, count, cfg in cases:
        print("static queue fit:", workload, count, cfg, flush=True)
        b = synth.make(workload, count=count)
        db = shape.DeviceBatch.from_host(b, "cuda:0")
        o = shape.default_opts()
        rec0, _, _ = shape.centroid(db, o)
        rec1, _, _ = shape.moments(db, rec0, o)
        c = shape.queue_cfg(**cfg)
        ref = shape.fit_queue(db, rec=rec1, opts=o, cfg=c, use_graph=False, want_perr=True)
        out = {k: torch.full_like(v, -7) for k, v in ref.items() if isinstance(v, torch.Tensor)}
        shape.fit_queue_static(db, rec=rec1, opts=o, cfg=c, out=out)
        torch.cuda.synchronize()
        for k in ("p", "chi2", "perr", "iters", "status", "sweeps"):
            np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k].cpu().numpy(), err_msg=k)
        conv = ((out["status"] & shape.ST_CONVERGED) != 0).float().mean().item()
        assert conv > 0.8, conv
