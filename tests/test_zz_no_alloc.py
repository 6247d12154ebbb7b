"""The fit entry point that allocates nothing (ckf_fit_noalloc: the fit's
records in the library's fixed per-GPU scratch array) against ckf_fit with a
caller workspace, both through the C ABI: identical outputs on two calls in
a row, the second with a smaller input, for both smoothers; a capacity
beyond the scratch limit fails with CKF_ERR_CAPACITY and writes nothing."""
import ctypes as C
import sys

import numpy as np
import pytest

from synth import make_event

pytestmark = pytest.mark.gpu
CKF_ERR_CAPACITY = 3  # include/ckf.h


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_fit_noalloc_equals_fit(det_dense):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22822_amd as ckf
    from paper_2505_22822_amd import _abi
    lib = _abi.load()
    geo = ckf.Geometry(det_dense.as_arrays())
    fld = ckf.UniformField(0, 0, 2.0)
    p = lambda t: C.c_void_p(t.data_ptr())
    limit = int(lib.ckf_fit_noalloc_max_meas())
    nb = C.c_size_t(0)
    assert lib.ckf_fit_workspace_size(limit, C.byref(nb)) == 0 and nb.value <= int(lib.ckf_fit_noalloc_max_bytes())
    assert lib.ckf_fit_workspace_size(limit + 1, C.byref(nb)) == 0 and nb.value > int(lib.ckf_fit_noalloc_max_bytes())
    sizes = []
    for seed, mu in ((41, 60), (42, 20)):  # the second call has the smaller input
        ev = make_event(det_dense, seed, mu=mu)
        b = ckf.Batch.from_event(ev)
        finder = ckf.Finder(geo, fld, b, ckf.config(), counters=False, meas_states=True)
        finder.enqueue()
        r = finder.result()
        nt, nm = r["n_tracks"], int(r["offsets"][r["n_tracks"]])
        sizes.append(nm)
        _say(f"[no-alloc] event {seed} mu {mu}: {nt} tracks, {nm} measurements (limit {limit})")
        assert 0 < nm <= limit
        t = finder.out
        for smoother in ("rts", "two_filter"):
            f = ckf.Fitter.from_finder(finder, smoother)
            f.enqueue()
            ref = f.result()
            params = torch.full((nm, 5), 7.0, dtype=torch.float64, device="cuda")
            cov = torch.full((nm, 15), 7.0, dtype=torch.float64, device="cuda")
            chi2 = torch.full((nt,), 7.0, dtype=torch.float64, device="cuda")
            ok = torch.full((nt,), 7, dtype=torch.int32, device="cuda")
            st = lib.ckf_fit_noalloc(geo.handle, fld.handle, C.byref(f._meas), C.byref(f._seeds), C.byref(f.cfg),
                                     p(t["n_tracks"]), nt, nm, p(t["offsets"]), p(t["meas"]), p(t["meas_surface"]),
                                     p(t["seed"]), f.smoother, p(params), p(cov), p(chi2), p(ok), None)
            assert st == 0, lib.ckf_last_error()
            torch.cuda.synchronize()
            assert np.array_equal(ok.cpu().numpy(), ref["ok"])
            assert np.all(ref["ok"] == 1)
            np.testing.assert_array_equal(params.cpu().numpy(), ref["params"])
            np.testing.assert_array_equal(cov.cpu().numpy(), ref["cov"])
            np.testing.assert_array_equal(chi2.cpu().numpy(), ref["chi2"])
            _say(f"  {smoother}: identical to ckf_fit")
    assert sizes[1] < sizes[0]
    # beyond the scratch limit: an error, and no output written
    f = ckf.Fitter.from_finder(finder, "rts")
    params = torch.full((4, 5), 7.0, dtype=torch.float64, device="cuda")
    st = lib.ckf_fit_noalloc(geo.handle, fld.handle, C.byref(f._meas), C.byref(f._seeds), C.byref(f.cfg),
                             p(t["n_tracks"]), 1, limit + 1, p(t["offsets"]), p(t["meas"]), p(t["meas_surface"]),
                             p(t["seed"]), 0, p(params), p(params), p(params), p(params), None)
    assert st == CKF_ERR_CAPACITY
    assert b"scratch" in lib.ckf_last_error()
    torch.cuda.synchronize()
    assert torch.all(params == 7.0)
