"""The C ABI library loads, exports every symbol include/ckf.h declares, and
rejects bad arguments on the host before touching the device (no GPU
needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "ckf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ckf_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2505_22822_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2505_22822_amd import build
        build.build()
    return _abi.load()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    from paper_2505_22822_amd import _abi
    assert set(names) == set(_abi.SIGNATURES), "binding and header disagree"


def test_struct_layouts_match_header(lib):
    """The ctypes mirrors have the sizes the C compiler gives the header's
    structs (checked by compiling a tiny probe with the host compiler)."""
    import subprocess
    import tempfile
    from paper_2505_22822_amd import _abi
    probe = r'''
#include <stdio.h>
#include "ckf.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(ckf_geometry_desc), sizeof(ckf_config), sizeof(ckf_measurements),
         sizeof(ckf_seeds), sizeof(ckf_tracks), sizeof(ckf_launch), sizeof(ckf_cells));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.c")
        open(src, "w").write(probe)
        exe = os.path.join(d, "p")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        sizes = [int(x) for x in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    mine = [C.sizeof(t) for t in (_abi.GeometryDesc, _abi.Config, _abi.Measurements, _abi.Seeds, _abi.Tracks,
                                  _abi.Launch, _abi.CellsDesc)]
    assert sizes == mine


def test_host_side_validation(lib):
    from paper_2505_22822_amd import _abi
    h = C.c_void_p()
    assert lib.ckf_geometry_create(None, C.byref(h)) == 1
    assert b"NULL" in lib.ckf_last_error()
    d = _abi.GeometryDesc()
    assert lib.ckf_geometry_create(C.byref(d), C.byref(h)) == 1  # empty
    assert lib.ckf_field_create_uniform(0.0, 0.0, float("nan"), C.byref(h)) == 1
    f = C.c_void_p()
    assert lib.ckf_field_create_uniform(0.0, 0.0, 2.0, C.byref(f)) == 0
    lib.ckf_field_destroy(f)
    cfg = _abi.Config()
    lib.ckf_config_default(C.byref(cfg))
    assert cfg.chi2_max == 15.0 and cfg.branches_per_surface == 3 and cfg.tracks_per_seed == 1
    assert cfg.learned_min_prob == 0.95 and cfg.learned_topk == 3
    nb = C.c_size_t(0)
    assert lib.ckf_workspace_size(None, C.byref(cfg), None, 1, 1, 1, C.byref(nb)) == 1
    assert lib.ckf_find(None, None, None, None, C.byref(cfg), None, None, None, 0, None, None) == 1
    assert lib.ckf_mlp_workspace_size(0, C.byref(nb)) == 1
    assert lib.ckf_capture_workspace_size(-1, C.byref(nb)) == 1
    assert lib.ckf_capture_workspace_size(0, C.byref(nb)) == 0
    small = nb.value
    assert lib.ckf_capture_workspace_size(600000, C.byref(nb)) == 0 and nb.value >= 600000 * 4 > small
    assert lib.ckf_capture_pairs(None, None, None, 0, None, None, None, 0, None, None, None, None, None, 0,
                                 None) == 1
    assert lib.ckf_model_create(None, None, C.byref(h)) == 1
    assert lib.ckf_mlp_adam(None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None) == 1
    assert lib.ckf_kf_update_batch(-1, None, None, None, None, None, None, None, None) == 1
    assert lib.ckf_status_string(5) == b"not supported"


def test_host_side_validation_of_the_next_rows(lib):
    """Argument checks of the fit, resolve, clustering and seeding entry
    points, taken on the host before any device work: NULL or negative
    arguments are rejected, sizes beyond the 32-bit index range are not
    supported, the workspace sizes grow with the problem, and the seeding
    top capacity accepts only [0, max]."""
    from paper_2505_22822_amd import _abi
    nb = C.c_size_t(0)
    # fit
    assert lib.ckf_fit_workspace_size(-1, C.byref(nb)) == 1
    assert lib.ckf_fit_workspace_size(0, C.byref(nb)) == 0
    small = nb.value
    assert lib.ckf_fit_workspace_size(10 ** 6, C.byref(nb)) == 0 and nb.value > small
    assert lib.ckf_fit(None, None, None, None, None, None, 0, 0, None, None, None, None, 0, None, 0, None, None, None,
                       None, None) == 1
    # ambiguity resolution
    assert lib.ckf_resolve_workspace_size(-1, 0, C.byref(nb)) == 1
    assert lib.ckf_resolve_workspace_size(10, 100, C.byref(nb)) == 0 and nb.value > 0
    assert lib.ckf_resolve(None, 5, 0, None, None, 0, None, None, 1, 8, None, 0, None, None, None) == 1  # NULL arrays
    assert lib.ckf_resolve(None, 0, 0, None, None, 0, None, None, -1, 8, None, 0, None, None, None) == 1  # max_shared < 0
    assert lib.ckf_resolve(None, 0, 0, None, None, 0, None, None, 1, 0, None, 0, None, None, None) == 1  # max_rounds 0
    assert lib.ckf_resolve(None, 0, 0, None, None, 1 << 31, None, None, 1, 8, None, 0, None, None, None) == 5
    # clustering
    cells = _abi.CellsDesc()
    assert lib.ckf_cluster_workspace_size(None, C.byref(nb)) == 1
    cells.n_events, cells.n_surfaces, cells.n_cells = -1, 10, 0
    assert lib.ckf_cluster_workspace_size(C.byref(cells), C.byref(nb)) == 1
    cells.n_events = 1
    assert lib.ckf_cluster_workspace_size(C.byref(cells), C.byref(nb)) == 0
    small = nb.value
    cells.n_cells = 10 ** 6
    assert lib.ckf_cluster_workspace_size(C.byref(cells), C.byref(nb)) == 0 and nb.value > small
    assert lib.ckf_cluster(None, C.byref(cells), None, None, 0, None, None, None, None, None, None, None) == 1
    # seeding
    assert lib.ckf_seed_workspace_size(1, 10, 0, 2, C.byref(nb)) == 1   # fewer than 3 layers
    assert lib.ckf_seed_workspace_size(1, 10, 0, 9, C.byref(nb)) == 1   # more than 8
    assert lib.ckf_seed_workspace_size(1, 10, 100, 4, C.byref(nb)) == 0
    small = nb.value
    assert lib.ckf_seed_workspace_size(2, 10, 100, 4, C.byref(nb)) == 0 and nb.value > small  # bins per event
    layers = (C.c_int32 * 4)(0, 1, 2, 3)
    n = C.c_int32(0)
    assert lib.ckf_seed(None, 1, None, 0, None, None, layers, 4, 2.0, None, 0, 0, C.byref(n), None, None, None, None,
                        None, None, None) == 1
    mx = C.c_int32(0)
    assert lib.ckf_seed_set_top_cap(-1, C.byref(mx)) == 1 and mx.value > 0
    assert lib.ckf_seed_set_top_cap(mx.value + 1, None) == 1
    assert lib.ckf_seed_set_top_cap(0, None) == 0
    assert lib.ckf_seed_set_top_cap(mx.value, None) == 0  # back to the default
