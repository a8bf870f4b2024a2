"""The interdigitated aperture selection without a workspace argument (its
dynamic-programming values in the library's static device array) gives the
same openings, prices and choice, bit for bit, as the workspace form, on two
calls in a row with the second smaller than the first."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _inputs(n_cp, n_rows, n_cols, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.standard_normal((n_cp, n_rows, n_cols)).astype(np.float32)
    p[:, :, : n_cols // 4] = 0.0                     # exact zero padding: ties
    occ = (rng.uniform(size=n_cp) < 0.3).astype(np.uint8)
    L = rng.integers(0, n_cols // 2, (n_cp, n_rows)).astype(np.int32)
    R = (L + rng.integers(0, n_cols // 2, (n_cp, n_rows))).astype(np.int32)
    return p, occ, L, R


def _run(dv, geom, p, occ, win, noalloc):
    dev = "cuda"
    n_cp, n_rows = geom.n_cp, geom.n_rows
    out = dict(L=torch.full((n_cp, n_rows), -7, dtype=torch.int32, device=dev),
               R=torch.full((n_cp, n_rows), -7, dtype=torch.int32, device=dev),
               cp_price=torch.full((n_cp,), -7.0, device=dev),
               best=torch.full((1,), -7, dtype=torch.int32, device=dev),
               best_price=torch.full((1,), -7.0, device=dev))
    ptrs = [dv._ptr(out[k]) for k in ("L", "R", "cp_price", "best", "best_price")]
    stream = dv._stream()
    if noalloc:
        code = dv.lib.dvmat_aperture_select_interdigitated_noalloc(geom, dv._ptr(p), dv._ptr(occ), dv._ptr(win),
                                                                   *ptrs, stream)
    else:
        nbytes = ctypes.c_size_t()
        assert dv.lib.dvmat_aperture_select_ws_size(geom, ctypes.byref(nbytes)) == 0
        ws = dv._workspace(nbytes.value, torch.device(dev))
        code = dv.lib.dvmat_aperture_select_interdigitated(geom, dv._ptr(p), dv._ptr(occ), dv._ptr(win), *ptrs,
                                                           dv._ptr(ws), ws.numel(), stream)
    assert code == 0, dv.lib.dvmat_last_error()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("windows", [False, True])
def test_noalloc_select_matches_workspace_form(windows):
    assert torch.cuda.is_available()
    from paper_1503_01721_amd import dvmat as dv
    # first the full-scale beamlet grid (180 x 40 x 40: 24.8 MB of state values),
    # then a smaller one that reuses the array with the first call's values in it
    for n_cp, n_rows, n_cols, seed in ((180, 40, 40, 11), (12, 5, 9, 12)):
        geom = dv.Geom(n_cp, n_rows, n_cols)
        p, occ, L, R = _inputs(n_cp, n_rows, n_cols, seed)
        pd, occd = torch.from_numpy(p).cuda(), torch.from_numpy(occ).cuda()
        win = None
        if windows:
            win = dv.leaf_windows(n_cp, n_rows, n_cols, occd, torch.from_numpy(L).cuda(),
                                  torch.from_numpy(R).cuda(), max(1, n_cols // 8))
        ref = _run(dv, geom, pd, occd, win, noalloc=False)
        got = _run(dv, geom, pd, occd, win, noalloc=True)
        for k in ref:
            assert np.array_equal(ref[k], got[k]), (n_cp, n_rows, n_cols, k)
        assert ref["best"][0] >= 0 and not occ[ref["best"][0]]
        assert (ref["cp_price"][occ == 1] == np.inf).all()
