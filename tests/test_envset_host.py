"""Host-side checks of the cached-environment set (no GPU): the workspace
query and create validate the grid and the substitution lists before any
device work (create touches no device memory), and the workspace holds the
2 (cols - 1) column environments."""
import ctypes as C

import numpy as np
import pytest

import paper_1908_08553_amd as tn
from paper_1908_08553_amd._native import tn_grid

lib = tn.lib


def lists(nets):
    counts = [len(n) for n in nets]
    flat = [i for n in nets for i in n]
    return ((C.c_int32 * max(len(counts), 1))(*counts), (C.c_int32 * max(len(flat), 1))(*flat),
            len(counts))


def workspace(rows, cols, D, nets, prec=tn.TN_PREC_F64):
    g = tn_grid(rows, cols, D, None, None)
    counts, flat, n = lists(nets)
    out = C.c_size_t()
    st = lib.tn_envset_workspace(C.byref(g), prec, n, counts, flat, C.byref(out))
    return st, out.value


def test_workspace_grows_with_environments():
    st, small = workspace(4, 2, 4, [[0]])
    assert st == tn.TN_OK and small > 0
    st, big = workspace(4, 8, 4, [[0]])
    assert st == tn.TN_OK
    # each of the 2 (cols - 1) environments keeps a one-column workspace
    # holding at least two boundaries of D^(rows+1) float64 entries
    assert big >= 2 * 7 * 2 * 4 ** 5 * 8
    st, f32 = workspace(4, 8, 4, [[0]], tn.TN_PREC_F32)
    assert st == tn.TN_OK and f32 < big


@pytest.mark.parametrize("nets", [[[-1]], [[12]], [[3, 3]], [[0, 5, 0]]])
def test_bad_substitutions_rejected(nets):
    st, _ = workspace(3, 4, 2, nets)
    assert st == tn.TN_EINVAL
    assert lib.tn_last_error()


def test_bad_grid_and_arguments_rejected():
    assert workspace(0, 4, 2, [[0]])[0] == tn.TN_EINVAL
    assert workspace(3, 3, 0, [[0]])[0] == tn.TN_EINVAL
    g = tn_grid(3, 3, 2, None, None)
    out = C.c_size_t()
    counts = (C.c_int32 * 1)(-1)
    assert lib.tn_envset_workspace(C.byref(g), 0, 1, counts, None, C.byref(out)) == tn.TN_EINVAL
    assert lib.tn_envset_workspace(C.byref(g), 7, 0, None, None, C.byref(out)) == tn.TN_EINVAL
    assert lib.tn_envset_workspace(None, 0, 0, None, None, C.byref(out)) == tn.TN_EINVAL
    # no networks: the base network alone
    assert lib.tn_envset_workspace(C.byref(g), 0, 0, None, None, C.byref(out)) == tn.TN_OK


def test_create_checks_workspace_without_touching_it():
    # one stream: create makes no streams or events, so it runs without a device
    lib.tn_set_option(tn.TN_OPT_ENV_STREAMS, 1)
    try:
        check_create()
    finally:
        lib.tn_set_option(tn.TN_OPT_ENV_STREAMS, 4)


def check_create():
    rows, cols, D = 3, 5, 2
    nets = [[0], [7], [2, 3]]
    st, need = workspace(rows, cols, D, nets)
    assert st == tn.TN_OK
    buf = np.zeros(need + 512, dtype=np.uint8)     # a stand-in address, never dereferenced
    base = buf.ctypes.data
    aligned = (base + 255) // 256 * 256
    g = tn_grid(rows, cols, D, None, None)
    counts, flat, n = lists(nets)
    h = C.c_void_p()
    assert lib.tn_envset_create(C.byref(g), 0, n, counts, flat, C.c_void_p(aligned), need - 256,
                                C.byref(h)) == tn.TN_ENOMEM
    assert lib.tn_envset_create(C.byref(g), 0, n, counts, flat, C.c_void_p(aligned + 8), need,
                                C.byref(h)) == tn.TN_EINVAL
    assert lib.tn_envset_create(C.byref(g), 0, n, counts, flat, C.c_void_p(aligned), need,
                                C.byref(h)) == tn.TN_OK
    assert h.value
    assert lib.tn_envset_destroy(h) == tn.TN_OK
    assert lib.tn_envset_destroy(None) == tn.TN_OK


def test_stream_option_range_and_workspace():
    assert lib.tn_set_option(tn.TN_OPT_ENV_STREAMS, 0) == tn.TN_EINVAL
    assert lib.tn_set_option(tn.TN_OPT_ENV_STREAMS, 5) == tn.TN_EINVAL
    try:
        sizes = []
        for s in (1, 2, 4):
            assert lib.tn_set_option(tn.TN_OPT_ENV_STREAMS, s) == tn.TN_OK
            sizes.append(workspace(4, 5, 3, [[0], [6]])[1])
        # each further stream adds one network region
        assert sizes[0] < sizes[1] < sizes[2]
        assert sizes[2] - sizes[1] == 2 * (sizes[1] - sizes[0])
    finally:
        lib.tn_set_option(tn.TN_OPT_ENV_STREAMS, 4)


def test_in_column_environments_budget():
    # environments inside columns add workspace only within the budget
    try:
        sizes = {}
        for gib in (0, 32):
            assert lib.tn_set_option(tn.TN_OPT_ENV_ROWS, gib) == tn.TN_OK
            sizes[gib] = workspace(6, 6, 4, [[0], [7], [8, 14]])[1]
        assert sizes[32] > sizes[0]
        assert lib.tn_set_option(tn.TN_OPT_ENV_ROWS, -1) == tn.TN_EINVAL
        assert lib.tn_set_option(tn.TN_OPT_ENV_ROWS, 2000) == tn.TN_EINVAL
        # 12 x 12 at D = 4 in float64 would add about 140 GiB: over the budget
        assert lib.tn_set_option(tn.TN_OPT_ENV_ROWS, 32) == tn.TN_OK
        big = workspace(12, 12, 4, [[0]])[1]
        assert lib.tn_set_option(tn.TN_OPT_ENV_ROWS, 0) == tn.TN_OK
        assert workspace(12, 12, 4, [[0]])[1] == big
    finally:
        lib.tn_set_option(tn.TN_OPT_ENV_ROWS, 32)
