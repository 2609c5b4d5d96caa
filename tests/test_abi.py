"""C-ABI contract on the CPU: the library loads, exports every declared symbol,
validates its inputs without touching a GPU, and its host plan (device = -1)
reproduces the oracle's tree, grids and preimages exactly (independent code)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hhffbp.h")

H = pytest.importorskip("paper_2506_23568_amd")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hhffbp_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = H.lib()
    names = _declared()
    assert "hhffbp_plan" in names and "hhffbp_image" in names
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", H.library_path()], capture_output=True,
                         text=True, check=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n


def test_probe_library_exports_its_entry_point():
    """The VALU issue-rate probe (bench.py --workload valu_probe) is built with the
    package and exports its one C entry point; invalid arguments are refused
    before any GPU call."""
    import ctypes

    from paper_2506_23568_amd import build_lib

    assert os.path.exists(build_lib.PROBE_LIB), "run __graft_entry__.build()"
    out = subprocess.run(["nm", "-D", "--defined-only", build_lib.PROBE_LIB], capture_output=True,
                         text=True, check=True).stdout
    assert re.search(r"\bT hhffbp_probe_valu\b", out)
    L = ctypes.CDLL(build_lib.PROBE_LIB)
    L.hhffbp_probe_valu.restype = ctypes.c_int
    r = ctypes.c_double(0.0)
    for mode, blocks, iters, reps in ((8, 1, 1, 1), (-1, 1, 1, 1), (0, 0, 1, 1), (0, 1, 0, 1),
                                      (0, 1, 1, 0)):
        assert L.hhffbp_probe_valu(mode, blocks, iters, reps, ctypes.c_void_p(1), None,
                                   ctypes.byref(r)) == -1
    assert L.hhffbp_probe_valu(0, 1, 1, 1, None, None, ctypes.byref(r)) == -1


def test_config_default_layout():
    c = H.binding.default_config()
    assert (c.mode, c.stages, c.merge_factor, c.interp_taps) == (0, 3, 4, 4)
    assert list(c.oversample) == [3.0, 3.0, 3.5]
    assert (c.range_kernel, c.range_taps, c.storage, c.device) == (0, 7, 0, 0)
    assert c.range_oversample == 2.0 and abs(c.position_slack - 5e-3) < 1e-15
    assert (c.interp_kernel, c.final_staging, c.root_grid, c.range_fused) == (0, 1, 0, 0)
    assert list(c.oversample_leaf) == [0.0, 0.0, 0.0]
    assert c.range_gemm == H.binding.RANGE_GEMMS["split_bf16"] == 0


def test_final_stage_bricks(small):
    """Voxel bricks of 4 x 8 x 8 for the final stage; with staging off no
    (brick, depth-1 node) pair has a box, with it on at most all of them."""
    import math
    on = H.Plan(*_args(small), stages=2, device=-1).info()
    off = H.Plan(*_args(small), stages=2, device=-1, final_staging=False).info()
    d = small.grid_dims
    assert on["final_bricks"] == math.ceil(d[0] / 4) * math.ceil(d[1] / 8) * math.ceil(d[2] / 8)
    assert off["final_bricks"] == on["final_bricks"] and off["final_boxed"] == 0
    assert 0 < on["final_boxed"] <= on["final_bricks"] * 4


def _args(w):
    return (w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims)


@pytest.mark.parametrize("change,status", [
    (dict(merge_factor=3), -1), (dict(interp_taps=5), -1), (dict(range_taps=11), -1),
    (dict(oversample=0.5), -1), (dict(stages=-9), -1),
    (dict(root_grid=True, mode="direct_rc"), -1), (dict(root_grid=True, stages=0), -1),
    (dict(range_fused=True), -1),  # the ES range kernel
    (dict(range_fused=True, range_kernel="linear", storage="f16"), -1),
    (dict(range_fused=True, range_kernel="linear", mode="direct_rc"), -1),
    (dict(oversample_leaf=0.5), -1), (dict(oversample_leaf=(2.0, 0.0, 2.0)), -1),
    (dict(oversample_leaf=9.0), -1),
    (dict(range_gemm=2), -1), (dict(range_gemm=-1), -1),
])
def test_invalid_configurations_are_rejected(small, change, status):
    kw = dict(device=-1)
    kw.update(change)
    with pytest.raises(H.HHFFBPError) as e:
        H.Plan(*_args(small), **kw)
    assert e.value.status == status


def test_range_gemm_form_is_reported(small):
    """hhffbp_plan_info.range_gemm_form (the last field of the struct: a wrong
    layout in the binding reads garbage there).  A host-only plan has no device
    LDS opt-in, so the split GEMM reports its register form; the float32 GEMM
    and the fused level-1 BP report their own values."""
    kw = dict(device=-1, range_kernel="linear", range_oversample=4.0, stages=2)
    assert H.Plan(*_args(small), **kw).info()["range_gemm_form"] == 1
    assert H.Plan(*_args(small), range_gemm="f32", **kw).info()["range_gemm_form"] == 0
    assert H.Plan(*_args(small), storage="f16", **kw).info()["range_gemm_form"] == 0
    assert H.Plan(*_args(small), range_fused=True, **kw).info()["range_gemm_form"] == -1


def test_exact_direct_mode_plans_on_the_host(small):
    """mode = direct_exact plans without stages; an unknown mode is rejected."""
    info = H.Plan(*_args(small), mode="direct_exact", device=-1).info()
    assert info["stages"] == 0 and info["leaf_pairs"] == small.n_pos * int(np.prod(small.grid_dims))
    c = H.binding.default_config()
    assert H.binding.MODES["direct_exact"] == 2


def test_aperture_weights_are_validated(small):
    """Non-finite weights are rejected at plan time, a wrong length by the binding."""
    w = np.ones(small.n_pos)
    H.Plan(*_args(small), device=-1, weights=w)
    w[5] = np.nan
    with pytest.raises(H.HHFFBPError) as e:
        H.Plan(*_args(small), device=-1, weights=w)
    assert e.value.status == -1
    with pytest.raises(ValueError):
        H.Plan(*_args(small), device=-1, weights=np.ones(3))


def test_unknown_storage_is_rejected(small):
    c = H.binding.default_config()
    pos = np.ascontiguousarray(small.positions)
    fr = np.ascontiguousarray(small.freqs_hz)
    c.n_pos, c.n_freq = pos.shape[0], fr.shape[0]
    c.positions = pos.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.freqs_hz = fr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for a in range(3):
        c.grid_origin[a], c.grid_pitch[a], c.grid_dims[a] = (small.grid_origin[a], small.grid_pitch[a],
                                                             small.grid_dims[a])
    c.device = -1
    h = ctypes.c_void_p()
    for st, want in ((7, -1), (1, 0), (2, 0)):
        c.storage = st
        assert H.lib().hhffbp_plan(ctypes.byref(c), ctypes.byref(h)) == want
        if want == 0:
            H.lib().hhffbp_plan_destroy(h)


def test_invalid_inputs_are_rejected(small):
    pos = small.positions.copy()
    pos[3, 1] = np.nan
    with pytest.raises(H.HHFFBPError) as e:
        H.Plan(pos, *_args(small)[1:], device=-1)
    assert e.value.status == -1
    behind = small.grid_origin.copy()
    behind[2] = -0.1
    with pytest.raises(H.HHFFBPError):
        H.Plan(small.positions, small.freqs_hz, behind, small.grid_pitch, small.grid_dims, device=-1)
    with pytest.raises(H.HHFFBPError):
        H.Plan(small.positions, small.freqs_hz[:1], *_args(small)[2:], device=-1)
    with pytest.raises(H.HHFFBPError):
        H.Plan(small.positions, np.full(4, 30e9), *_args(small)[2:], device=-1)
    L = H.lib()
    h = ctypes.c_void_p()
    assert L.hhffbp_plan(None, ctypes.byref(h)) == -1
    assert b"NULL" in L.hhffbp_last_error()


def test_host_only_plan_refuses_image(small):
    pl = H.Plan(*_args(small), stages=1, device=-1)
    assert pl.workspace_bytes() > 0
    L = H.lib()
    assert L.hhffbp_image(pl._h, 1, None, 1, 256, 1 << 30, None) == -4
    with pytest.raises(H.HHFFBPError):
        pl.node_layout(0, 0)
    with pytest.raises(H.HHFFBPError):
        pl.node_layout(2, 0)


@pytest.mark.parametrize("S,Q,gamma,T,root,leaf", [
    (1, 4, 3.0, 4, False, None), (2, 4, 3.0, 4, False, None), (2, 2, (2.5, 2.5, 3.0), 6, False, None),
    (1, 4, 3.0, 4, True, None), (2, 2, (2.5, 2.5, 3.0), 4, True, None),
    (2, 4, (2.2, 2.2, 2.6), 4, False, (1.8, 1.8, 2.2)), (2, 4, (2.2, 2.2, 2.6), 4, True, (1.8, 1.8, 2.2)),
])
def test_host_plan_matches_oracle_plan(small, S, Q, gamma, T, root, leaf):
    from oracle import plan as OP

    pl = H.Plan(*_args(small), stages=S, merge_factor=Q, oversample=gamma, interp_taps=T,
                device=-1, root_grid=root, oversample_leaf=leaf)
    op = OP.build_plan(*_args(small), S, Q, gamma, T, root_grid=root, gamma_leaf=leaf)
    info = pl.info()
    assert info["n_leaves"] == sum(1 for n in op.levels[S] if not n.empty)
    assert info["root_grid"] == int(root)
    if root:
        assert info["level_points"][0] == op.levels[0][0].lattice.size
        assert info["final_pairs"] == int(np.prod(small.grid_dims))
    for d in range(0 if root else 1, S + 1):
        for i, node in enumerate(op.levels[d]):
            lay = pl.node_layout(d, i)
            if node.empty:
                assert lay["npoints"] == 0
                continue
            L = node.lattice
            assert (lay["i0"], lay["j0"], lay["ni"], lay["nj"]) == (L.i0, L.j0, L.ni, L.nj)
            assert np.array_equal(lay["l_lo"], L.l_lo) and np.array_equal(lay["l_hi"], L.l_hi)
            assert np.array_equal(lay["off"], L.off)
            xyz = pl.node_points(d, i)
            assert np.array_equal(np.isfinite(xyz[:, 2]), L.valid)
            assert np.max(np.abs(xyz[L.valid] - L.xyz[L.valid])) < 1e-12


def test_reductions_validate_without_a_gpu():
    L = H.lib()
    nb = ctypes.c_size_t()
    assert L.hhffbp_stats_workspace_bytes(ctypes.byref(nb)) == 0 and nb.value == 1024 * 8 * 8
    assert L.hhffbp_stats_workspace_bytes(None) == -1
    dummy = ctypes.c_void_p(256)  # never dereferenced: every call below fails validation first
    assert L.hhffbp_image_stats(None, None, 10, dummy, dummy, nb.value, None) == -1
    assert L.hhffbp_image_stats(dummy, None, -1, dummy, dummy, nb.value, None) == -1
    assert L.hhffbp_image_stats(dummy, None, 10, dummy, None, nb.value, None) == -5
    assert L.hhffbp_image_stats(dummy, None, 10, dummy, dummy, nb.value - 8, None) == -5
    assert L.hhffbp_loss_grad(dummy, None, 10, None, 1.0, 1.0, dummy, dummy, None) == -1
    assert L.hhffbp_loss_grad(dummy, None, -3, dummy, 1.0, 1.0, dummy, dummy, None) == -1
    assert L.hhffbp_loss_grad(dummy, None, 10, dummy, float("nan"), 1.0, dummy, dummy, None) == -1
    dims = (ctypes.c_int64 * 3)(4, 0, 4)
    assert L.hhffbp_box_peaks(dummy, ctypes.byref(dims), 1, dummy, dummy, None) == -1
    dims = (ctypes.c_int64 * 3)(4, 4, 4)
    assert L.hhffbp_box_peaks(dummy, ctypes.byref(dims), -1, dummy, dummy, None) == -1
    assert L.hhffbp_box_peaks(None, ctypes.byref(dims), 2, dummy, dummy, None) == -1
    assert b"box_peaks" in L.hhffbp_last_error()


def test_automatic_stages_minimise_the_cost_model(small):
    """stages = -K picks the S in 1..K with the smallest Sec. IV-B operation
    count (model_ms) among host plans built for each S; invalid forms fail."""
    for rk, U, root in (("es", 2.0, False), ("linear", 8.0, False), ("linear", 8.0, True)):
        kw = dict(range_kernel=rk, range_oversample=U, device=-1, root_grid=root)
        costs = [H.Plan(*_args(small), stages=s, **kw).info()["model_ms"] for s in (1, 2, 3)]
        auto = H.Plan(*_args(small), stages=-3, **kw).info()
        assert auto["stages"] == 1 + int(np.argmin(costs))
        assert abs(auto["model_ms"] - min(costs)) <= 1e-12 + 1e-9 * min(costs)
        assert all(c > 0 for c in costs)
    with pytest.raises(H.HHFFBPError):
        H.Plan(*_args(small), stages=-2, mode="direct_rc", device=-1)
    with pytest.raises(H.HHFFBPError):
        H.Plan(*_args(small), stages=-9, device=-1)


def test_host_only_plan_refuses_images(small):
    """A host-only plan (device = -1) holds no device tables: hhffbp_image and
    hhffbp_image_noalloc return HHFFBP_E_DEVICE before touching a GPU."""
    pl = H.Plan(*_args(small), stages=2, device=-1)
    L = H.lib()
    dummy = ctypes.c_void_p(256)  # never dereferenced: the calls stop at the plan check
    st = L.hhffbp_image_noalloc(pl._h, dummy, None, dummy, None)
    assert st == -4 and b"host-only" in L.hhffbp_last_error()
    st = L.hhffbp_image(pl._h, dummy, None, dummy, dummy, 1 << 30, None)
    assert st == -4
