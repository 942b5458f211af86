"""GPU tests of the request server (continuous batching of solves).

Each request's result must be the same alone and in the mix: the server runs
the same kernels with per-request, fixed-order reductions on its own stream,
so the results are compared bit for bit with a standalone nps_solve, and
judged on the oracle's FP64 true residual.
"""
import time

import numpy as np
import pytest
import torch

import nps_inputs as gi
from oracle import laplacian as lap

pytestmark = pytest.mark.gpu

nps = pytest.importorskip("paper_2310_00177_amd")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def scene(n, seed):
    spec = gi.scene_c1() if n == 32 else gi.scene_serving(n)
    lab = gi.gen_labels(spec, seed=seed)
    return lab, gi.gen_rhs(lab, seed=seed + 1)


def drain(srv, ids, timeout_s=90.0):
    out, peak = {}, 0
    t0 = time.time()
    while len(out) < len(ids):
        active, _ = srv.step()
        peak = max(peak, active)
        for rid in ids:
            if rid not in out:
                r = srv.poll(rid)
                if r is not None:
                    out[rid] = r
        assert time.time() - t0 < timeout_s, "server did not finish"
    return out, peak


@pytest.fixture(scope="module")
def net():
    return nps.Net(gi.multilevel_params(6), 6)


@pytest.mark.parametrize("precision", [nps.MIXED_BF16, nps.FP32])
def test_results_in_the_mix_equal_standalone(net, precision):
    reqs = [scene(n, 40 + i) for i, n in enumerate([64, 32, 96, 64, 128, 32])]
    srv = nps.Server(net, hbm_budget=4 << 30, max_slots=4)
    ids = [srv.submit(lab, b, precision=precision) for lab, b in reqs]
    print(f"submitted {len(ids)} requests", flush=True)
    res, peak = drain(srv, ids)
    assert peak >= 2, "requests never overlapped"
    for (lab, b), rid in zip(reqs, ids):
        x, info, lat = res[rid]
        xs, infos = nps.solve(net, torch.from_numpy(lab).cuda(), torch.from_numpy(b).cuda(), precision=precision)
        assert info.status == 0 and info.iterations == infos.iterations
        np.testing.assert_array_equal(x, xs.cpu().numpy())
        assert lap.rel_residual(lab, b, x) < 1e-6
        assert lat > 0.0
    srv.close()


def test_tight_budget_forces_queueing(net):
    reqs = [scene(64, 60 + i) for i in range(3)]
    srv = nps.Server(net, hbm_budget=srv_bytes(net, (64, 64, 64)) + (1 << 20), max_slots=4)
    ids = [srv.submit(lab, b) for lab, b in reqs]
    res, peak = drain(srv, ids)
    assert peak == 1
    for (lab, b), rid in zip(reqs, ids):
        assert res[rid][1].status == 0 and lap.rel_residual(lab, b, res[rid][0]) < 1e-6
    srv.close()


def srv_bytes(net, shape):
    probe = nps.Server(net, hbm_budget=1 << 24, max_slots=1)
    nbytes = probe.request_bytes(shape)
    probe.close()
    return nbytes


def test_bad_request_fails_alone(net):
    good, bad = scene(32, 70), scene(32, 71)
    lab_bad = bad[0].copy()
    lab_bad[5, 5, 5] = 9
    srv = nps.Server(net, hbm_budget=1 << 30, max_slots=2)
    ids = [srv.submit(good[0], good[1]), srv.submit(lab_bad, bad[1])]
    assert srv.poll(ids[0]) is None   # pending before any step
    res, _ = drain(srv, ids)
    assert res[ids[0]][1].status == 0
    assert res[ids[1]][1].status == -3
    assert res[ids[1]][0] is None   # a rejected request returns no solution
    with pytest.raises(nps.NpsError):
        srv.submit(good[0][:, :, :16].copy(), good[1][:, :, :16].copy())   # 16 % 32
    srv.close()
