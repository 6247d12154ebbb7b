"""Stream ordering of the binding: buffers a binding object allocates are
zero-filled on torch's current stream, and the library's calls run on the
stream the caller names.  The objects wait for their fills, so a call
enqueued at once on another stream sees complete buffers (regression test:
a fit's output flags were once zeroed by a fill still pending on the other
stream)."""
import sys

import numpy as np
import pytest

from synth import make_event

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ckf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2505_22822_amd as ckf
    return ckf


def test_calls_on_another_stream_see_complete_buffers(ckf, det_dense):
    """With torch's current stream held busy by a bounded spin kernel while
    a finder and a fitter are made, their calls enqueued at once on a second
    stream return the same tracks and fits as calls on the current stream."""
    import torch
    ev = make_event(det_dense, 12, mu=20)
    geo = ckf.Geometry(det_dense.as_arrays())
    fld = ckf.UniformField(0, 0, 2.0)
    b = ckf.Batch.from_event(ev)
    ref_f = ckf.Finder(geo, fld, b, counters=False, meas_states=True)
    ref_f.enqueue()
    ref = ref_f.result()
    ref_fit = ckf.Fitter.from_finder(ref_f, "rts")
    ref_fit.enqueue()
    ref_g = ref_fit.result()
    _say(f"# streams: {ev.n_seeds} seeds, {ref['n_tracks']} tracks")
    s = torch.cuda.Stream()
    torch.cuda._sleep(20_000_000)  # a bounded spin on the current stream
    f = ckf.Finder(geo, fld, b, counters=False, meas_states=True)
    f.enqueue(s)
    got = f.result()
    assert got["n_tracks"] == ref["n_tracks"] > 0
    for k in ("offsets", "meas", "params", "cov", "seed"):
        assert np.array_equal(got[k], ref[k]), k
    torch.cuda._sleep(20_000_000)
    fit = ckf.Fitter.from_finder(f, "rts")
    fit.enqueue(s)
    g = fit.result()
    assert g["n_tracks"] == ref_g["n_tracks"] and np.all(g["ok"] == 1)
    assert np.array_equal(g["params"], ref_g["params"]) and np.array_equal(g["cov"], ref_g["cov"])
