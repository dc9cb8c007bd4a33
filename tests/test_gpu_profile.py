"""Kernel timing of pic_step (measurement support): the sampling stride
brackets only the steps k = 0, every, 2 every, ... of each call, and timing
leaves the steps' results unchanged, bit for bit."""
import numpy as np
import pytest

from paper_1906_08125_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1906_08125_amd import pic as P
    P.load_library()
    return P


def _run(pic, gm, cfg, n_steps, timing):
    """Two calls of n_steps each from the empty gap; timing: None, or the
    (every, expected push launches) of each call."""
    gs = pic.State(gm, 60_000)
    gs.init_field(cfg.E0, tol=cfg.tol)
    rate, _ = gm.emission_rate(gs.E, cfg.phi_w)
    # some 300 superparticles injected per step
    w_sp = float(rate) * cfg.dt / 300.0
    kw = dict(dt=cfg.dt, E0=cfg.E0, w_sp=w_sp, phi_w=cfg.phi_w,
              seed=cfg.seed, tol=cfg.tol, resort_every=4)
    rows = []
    for c in range(2):
        if timing:
            gm.profile(True, classes=("push",), every=timing[c][0])
        st = gs.step(step0=c * n_steps, n_steps=n_steps, **kw)
        torch.cuda.synchronize()
        if timing:
            kt = gm.profile_read()
            gm.profile(False)
            assert kt["push"]["launches"] == timing[c][1], (c, kt)
            assert kt["push"]["ms"] > 0.0
        rows += pic.State.decode_stats(st)
    out = {k: getattr(gs, k).cpu().numpy().copy()
           for k in ("x", "y", "z", "tet", "phi", "E", "charge", "n_slots")}
    return rows, out


def test_profile_stride_and_no_effect_on_results(pic):
    cfg = W.config_tiny()
    gm = pic.Mesh(cfg.mesh(), cfg.emit_zmin)
    # steps 0..5 timed every step (6 pushes); steps 6..11 every third step
    # (6 and 9: 2 pushes)
    rows_t, out_t = _run(pic, gm, cfg, 6, [(1, 6), (3, 2)])
    rows_u, out_u = _run(pic, gm, cfg, 6, None)
    assert len(rows_t) == len(rows_u) == 12
    for a, b in zip(rows_t, rows_u):
        assert a == b
    assert int(out_t["n_slots"][0]) > 0
    for k in out_t:
        assert np.array_equal(out_t[k], out_u[k]), k


def test_profile_every_rejects_below_one(pic):
    cfg = W.config_tiny()
    gm = pic.Mesh(cfg.mesh(), cfg.emit_zmin)
    with pytest.raises(Exception):
        gm.profile(True, classes=("push",), every=0)
    # the handle still times every step afterwards
    gm.profile(True, classes=("push",))
    gm.profile(False)
