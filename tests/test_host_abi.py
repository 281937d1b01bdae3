"""CPU checks of the C ABI: the library loads, exports every declared entry
point, sizes workspaces and rejects invalid arguments, without touching a GPU
(no compute call is made)."""
import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

from paper_2510_09204_amd import EXPORTED, load_library
from paper_2510_09204_amd.binding import SFConfigC
from workloads import WORKLOADS, make_batch, make_problem, pack

ROOT = Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def lib():
    return load_library()


def _declared():
    text = (ROOT / "include" / "sf.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sf_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert set(names) == set(EXPORTED)
    for name in names:
        assert getattr(lib, name) is not None


def _setup(lib, cfg, n, M, a, box, ws=None, nbytes=None):
    n = np.ascontiguousarray(n, dtype=np.int32)
    M = np.ascontiguousarray(M, dtype=np.int32)
    a = np.ascontiguousarray(a, dtype=np.float32)
    box = np.ascontiguousarray(box, dtype=np.float32)
    nb = ctypes.c_size_t(0 if nbytes is None else nbytes)
    plan = ctypes.c_void_p()
    rc = lib.sf_setup(ctypes.byref(cfg), len(n), n.ctypes.data, M.ctypes.data, a.ctypes.data,
                      box.ctypes.data, ws, ctypes.byref(nb), None, ctypes.byref(plan))
    return rc, nb.value, lib.sf_last_error_detail().decode()


def _cfg(**kw):
    base = dict(n_dim=2, n_coef=11, n_steps=100, checkpoint_every=10, max_iters=200,
                threads=0, rho=0.5)
    base.update(kw)
    return SFConfigC(**base)


BOX = [[[-5.8, -5.8], [5.8, 5.8]]]


def test_workspace_size_query(lib):
    rc, nbytes, _ = _setup(lib, _cfg(), [32], [20], [0.4], BOX)
    assert rc == 0
    S = 2 * 32 * 11
    # checkpoints (20 of (xi_bar, lambda)) + final state + 10-iterate recompute area
    assert nbytes >= 4 * S * (2 * 20 + 2 + 2 * 10)
    rc2, more, _ = _setup(lib, _cfg(max_iters=2000), [32], [20], [0.4], BOX)
    assert rc2 == 0 and more > nbytes


def test_workspace_size_for_uneven_batch(lib):
    probs = make_batch(WORKLOADS[4])
    pk = pack(probs)
    rc, nbytes, _ = _setup(lib, _cfg(max_iters=150), pk.n_robots, pk.n_obs, pk.robot_a, pk.box)
    assert rc == 0 and nbytes > 0


@pytest.mark.parametrize("kw,code", [
    (dict(n_dim=4), -2), (dict(n_dim=1), -2), (dict(n_coef=1), -2), (dict(n_coef=33), -2), (dict(n_steps=1), -2),
    (dict(rho=0.0), -1), (dict(rho=float("nan")), -1), (dict(threads=300), -1),
    (dict(checkpoint_every=0), -1), (dict(max_iters=-1), -1)])
def test_invalid_config_is_rejected(lib, kw, code):
    rc, _, detail = _setup(lib, _cfg(**kw), [4], [3], [0.3], BOX)
    assert rc == code and detail


@pytest.mark.parametrize("n,M,a,box,code", [
    ([0], [3], [0.3], BOX, -2), ([2000], [3], [0.3], BOX, -2), ([65], [3], [0.3], BOX, -2),
    ([4], [-1], [0.3], BOX, -2),
    ([4], [3], [0.0], BOX, -1), ([4], [3], [0.3], [[[1.0, -1.0], [0.0, 1.0]]], -1),
    ([4], [3], [0.3], [[[float("nan"), -1.0], [1.0, 1.0]]], -6)])
def test_invalid_problem_is_rejected(lib, n, M, a, box, code):
    """Counts, sizes and boxes outside the documented ranges (planar problems
    hold at most 64 robots: the update tiles cover 4 row tiles of 16)."""
    rc, _, detail = _setup(lib, _cfg(), n, M, a, box)
    assert rc == code and detail


BOX3 = [[[-5.8, -5.8, -2.7], [5.8, 5.8, 2.7]]]


def test_3d_workspace_size_query(lib):
    """n_dim = 3: robot sizes (a, b) per problem, box [2][3]; coefficient
    arrays hold three axes."""
    rc, nbytes, detail = _setup(lib, _cfg(n_dim=3, max_iters=0), [32], [20], [[0.4, 0.6]], BOX3)
    assert rc == 0, detail
    assert nbytes >= 4 * 3 * 32 * 11 * 5          # coefficient-sized areas of three axes


@pytest.mark.parametrize("a,box,code", [
    ([[0.4, 0.0]], BOX3, -1), ([[0.4, float("inf")]], BOX3, -1),
    ([[0.4, 0.6]], [[[-1.0, -1.0, 1.0], [1.0, 1.0, -1.0]]], -1),
    ([[0.4, 0.6]], [[[-1.0, -1.0, float("nan")], [1.0, 1.0, 1.0]]], -6)])
def test_invalid_3d_problem_is_rejected(lib, a, box, code):
    rc, _, detail = _setup(lib, _cfg(n_dim=3), [4], [3], a, box)
    assert rc == code and detail


def test_3d_state_too_large_for_lds_is_a_shape_error(lib):
    rc, _, detail = _setup(lib, _cfg(n_dim=3, n_coef=32, n_steps=100), [512], [0],
                           [[0.3, 0.3]], BOX3)
    assert rc == -2 and "LDS" in detail


def test_state_too_large_for_lds_is_a_shape_error(lib):
    rc, _, detail = _setup(lib, _cfg(n_coef=32, n_steps=4096), [64], [0], [0.3], BOX)
    assert rc == -2 and "LDS" in detail


def test_empty_batch_and_null_pointers(lib):
    cfg = _cfg()
    nb = ctypes.c_size_t(0)
    assert lib.sf_setup(ctypes.byref(cfg), 0, None, None, None, None, None,
                        ctypes.byref(nb), None, None) == -1
    assert lib.sf_setup(None, 1, None, None, None, None, None, ctypes.byref(nb), None,
                        None) == -1
    assert lib.sf_setup(ctypes.byref(cfg), 1, None, None, None, None, None, None, None,
                        None) == -1


def test_calls_without_plan_fail_cleanly(lib):
    assert lib.sf_project(None, None, None, None, None, None, None, 10, 0, None, None, None,
                          None) == -1
    assert lib.sf_project_backward(None, None, None, None, None, 0.0, None, None, None,
                                   None) == -1
    assert lib.sf_project_backward_static(None, None, None, None, None, 0.0, None, None,
                                          None, None) == -1
    lib.sf_destroy(None)
    assert lib.sf_plan_threads(None) == 0
    assert lib.sf_forward_generation(None) == -1
    assert lib.sf_set_early_exit(None, 1e-3, 10) == -1
    assert lib.sf_project_iterations(None, None, None, None) == -1
    assert lib.sf_smoothness(None, None, None, 5.0, None, None) == -1


def test_selection_calls_validate_before_launching(lib):
    """Argument checks of the selection entry points (no pointer is touched
    and nothing is launched when they fail)."""
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails its checks
    assert lib.sf_rank_residual(None, 4, 2, fake, None) == -1
    assert lib.sf_rank_residual(fake, 0, 1, fake, None) == -2
    assert lib.sf_rank_residual(fake, 9000, 1, fake, None) == -2
    assert lib.sf_rank_residual(fake, 4, 5, fake, None) == -1
    assert lib.sf_rank_residual(fake, 4, 0, fake, None) == -1
    assert lib.sf_select_best(fake, None, 4, 1e-3, fake, None) == -1
    assert lib.sf_select_best(fake, fake, 4, -1.0, fake, None) == -1
    assert lib.sf_select_best(fake, fake, 4, float("nan"), fake, None) == -1
    assert lib.sf_gather_blocks(fake, 4, None, 2, 8, fake, None) == -1
    assert lib.sf_gather_blocks(fake, 4, fake, 0, 8, fake, None) == -1
    assert lib.sf_gather_blocks(fake, 4, fake, 70000, 8, fake, None) == -1


def test_error_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.sf_error_string(code).decode()
    assert b"unknown" in lib.sf_error_string(-99)


def test_generator_is_deterministic_and_well_formed():
    cfg = WORKLOADS[3]
    a, b = make_problem(cfg, 5), make_problem(cfg, 5)
    np.testing.assert_array_equal(a.xi, b.xi)
    np.testing.assert_array_equal(a.obstacles, b.obstacles)
    pts = np.concatenate([a.boundary[:, 0], a.boundary[:, 1]])
    # obstacles clear of every start and goal
    for c in a.obstacles:
        assert np.min(np.hypot(*(pts - c[:2]).T)) > c[2]
    # starts (and goals) mutually separated, inside the box
    for k in range(2):
        P = a.boundary[:, k]
        d = np.hypot(*(P[:, None] - P[None]).transpose(2, 0, 1))
        assert np.min(d + 1e9 * np.eye(len(P))) >= 0.5
        assert np.all(np.abs(P) <= a.box[1, 0])
    # the noise-free trajectory interpolates the boundary
    np.testing.assert_allclose(a.straight[:, :, 0].T, a.boundary[:, 0], atol=1e-12)
    np.testing.assert_allclose(a.straight[:, :, -1].T, a.boundary[:, 1], atol=1e-12)


def test_candidates_share_their_context():
    cfg = WORKLOADS[2]
    ps = make_batch(cfg, batch=3)
    np.testing.assert_array_equal(ps[0].obstacles, ps[2].obstacles)
    np.testing.assert_array_equal(ps[0].boundary, ps[1].boundary)
    assert not np.array_equal(ps[0].xi, ps[1].xi)


def test_uneven_workload_ranges():
    ps = make_batch(WORKLOADS[4])
    ns = np.array([p.n for p in ps])
    Ms = np.array([p.M for p in ps])
    assert ns.min() >= 8 and ns.max() <= 64 and Ms.min() >= 0 and Ms.max() <= 30
    assert len(set(ns)) > 10
