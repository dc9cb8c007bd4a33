"""locate_noalloc, the entry point that allocates nothing: through the C
ABI, two calls in a row (the second with fewer points, so that a queue
counter left over from the first call would corrupt it), each compared bit
for bit with locate on the same points and hints."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1906_08125_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1906_08125_amd import pic as P
    P.load_library()
    return P


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _call(pic, fn, gm, pts, hint):
    x, y, z = (_dev(pts[:, k].copy()) for k in range(3))
    tet = _dev(hint.astype(np.int32))
    where = torch.full((len(pts),), 255, dtype=torch.uint8, device="cuda")
    st = fn(gm.handle, len(pts), C.c_void_p(x.data_ptr()),
            C.c_void_p(y.data_ptr()), C.c_void_p(z.data_ptr()),
            C.c_void_p(tet.data_ptr()), C.c_void_p(where.data_ptr()),
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == pic.PIC_OK, pic.load_library().pic_last_error()
    torch.cuda.synchronize()
    return tet.cpu().numpy(), where.cpu().numpy()


def test_locate_noalloc_matches_locate(pic):
    L = pic.load_library()
    cfg = W.config_tiny()
    tip = cfg.mesh()
    gm = pic.Mesh(tip, cfg.emit_zmin)
    rng = np.random.default_rng(11)
    cases = []
    # first call: 300k points with mixed hints (random tets and none)
    p1 = np.concatenate([W.random_points_in_box(tip, 290_000, 21),
                         W.lattice_points(tip, 10_000, 22)])
    h1 = np.where(rng.random(len(p1)) < 0.5, rng.integers(0, gm.n_tets, len(p1)), -1)
    cases.append((p1, h1))
    # second call: fewer points, none hinted (all through the exact scan)
    p2 = W.random_points_in_box(tip, 60_000, 23)
    cases.append((p2, np.full(len(p2), -1)))
    for pts, hint in cases:
        t_ref, w_ref = _call(pic, L.locate, gm, pts, hint)
        t_na, w_na = _call(pic, L.locate_noalloc, gm, pts, hint)
        print(len(pts), "inside", int((w_ref == 0).sum()), "anode",
              int((w_ref == 1).sum()), "outside", int((w_ref == 2).sum()))
        assert (w_ref != 255).all()
        assert np.array_equal(t_na, t_ref)
        assert np.array_equal(w_na, w_ref)
    gm.close()


def test_locate_noalloc_rejects_beyond_maximum(pic):
    L = pic.load_library()
    cfg = W.config_tiny()
    gm = pic.Mesh(cfg.mesh(), cfg.emit_zmin)
    st = L.locate_noalloc(gm.handle, pic.LOCATE_NOALLOC_MAX + 1, None, None,
                          None, None, None, None)
    assert st == pic.PIC_E_ARG
    assert b"PIC_LOCATE_NOALLOC_MAX" in L.pic_last_error()
    gm.close()
