"""GPU sign from local BHM weights (eq. sign_prediction) and the threshold update
(eq. online_surf_logodds) against the oracle, on synthetic weights for the small room.
Double points: log-odds within 1e-12 (FP64, a different summation order: the GPU
separates the RBF by axis).  Float points (FP32 arithmetic with a compensated outer
sum): log-odds within 100 float roundings of sum |w_h k(x, h)| (the FP32 exp and the
products and inner sums carry a few roundings each).  Signs identical wherever |l - tau|
exceeds the tolerance, and the sign feeding a query."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_29227_amd import ksdf, scenes
from tests.bhm_bound import abs_terms

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _setup(hinges=7):
    wl = scenes.small_room_workload(n_queries=20000)
    b = scenes.bhm_weights(wl, hinges=hinges)
    rng = np.random.default_rng(3)
    near = wl.points[rng.choice(len(wl.points), 20000)] + rng.normal(0, 0.02, (20000, 3))
    q = np.concatenate([near, wl.queries.astype(np.float64)])
    return wl, b, q


def _args(b):
    return (b["origin"], b["box"], b["dims"], b["hinges"], b["gamma"],
            torch.from_numpy(b["box_bhm"]).cuda(), torch.from_numpy(b["weights"]).cuda())


@pytest.mark.parametrize("dtype,hinges", [(torch.float64, 7), (torch.float32, 7), (torch.float32, 5)])
def test_bhm_sign_matches_oracle(dtype, hinges):
    """7 hinges per axis runs the FP32 form unrolled for that count; 5 the general one."""
    _say(f"bhm sign {dtype}, {hinges} hinges per axis")
    wl, b, q = _setup(hinges)
    qt = torch.from_numpy(q).to("cuda", dtype)
    qd = qt.double().cpu().numpy()
    for tau in (0.0, 0.3):
        sign, lo = ksdf.bhm_sign(qt, *_args(b), tau=tau, logodds=True)
        torch.cuda.synchronize()
        olo, have, osign = oracle.bhm(qd, b["origin"], b["box"], b["dims"], b["hinges"],
                                      b["gamma"], b["box_bhm"], b["weights"], tau=tau)
        g = lo.cpu().numpy()
        h = have == 1
        assert np.all(np.isneginf(g[~h]))
        tol = 1e-12 if dtype == torch.float64 else 100 * 2.0 ** -24 * abs_terms(qd, b)
        err = np.abs(g[h] - olo[h])
        print(f"bhm {dtype} tau {tau}: max |dl| {err.max():.3g}, max |dl| / tol "
              f"{(err / np.broadcast_to(tol, g.shape)[h]).max():.3g}", flush=True)
        assert np.all(err <= np.broadcast_to(tol, g.shape)[h])
        s = sign.cpu().numpy().astype(np.int32)
        clear = ~h | (np.abs(olo - tau) > tol)
        print(f"ambiguous signs: {int((~clear).sum())} of {len(s)}", flush=True)
        assert np.array_equal(s[clear], osign[clear])
        assert h.mean() > 0.3 and (osign == -1).any() and (osign == 1).any()


def test_bhm_tau_update_and_query_sign():
    _say("bhm tau update, sign into a query")
    wl, b, q = _setup()
    hits = torch.from_numpy(np.asarray(wl.points[:5000], np.float32)).cuda()
    tau = torch.tensor([0.4], dtype=torch.float64, device="cuda")
    ksdf.bhm_update_tau(hits, *_args(b), 0.25, tau)
    torch.cuda.synchronize()
    olo, _, _ = oracle.bhm(hits.double().cpu().numpy(), b["origin"], b["box"], b["dims"],
                           b["hinges"], b["gamma"], b["box_bhm"], b["weights"])
    # float hits: FP32 log-odds (tolerance as above), summed in float-float
    tol = 100 * 2.0 ** -24 * abs_terms(hits.double().cpu().numpy(), b).mean() * 0.25 + 1e-12
    assert float(tau.item()) == pytest.approx(oracle.bhm_update_tau(0.4, olo, 0.25), abs=tol)
    tau64 = torch.tensor([0.4], dtype=torch.float64, device="cuda")
    ksdf.bhm_update_tau(hits.double(), *_args(b), 0.25, tau64)
    torch.cuda.synchronize()
    assert float(tau64.item()) == pytest.approx(oracle.bhm_update_tau(0.4, olo, 0.25), abs=1e-12)
    # the sign goes straight into the query: d = s u
    cells = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min)
    model = ksdf.Model(cells, len(wl.points), wl.origin, wl.h, ell=wl.ell, noise_var=wl.noise_var)
    model.fit(torch.from_numpy(wl.points).cuda())
    qt = torch.from_numpy(wl.queries).cuda()
    sign = ksdf.bhm_sign(qt, *_args(b), tau=float(tau.item()))
    out = model.query(qt, sign)
    plain = model.query(qt)
    torch.cuda.synchronize()
    assert torch.equal(out["mean"], plain["mean"] * sign.float())
    model.close()
