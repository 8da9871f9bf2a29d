"""tn_set_option range checks (host only, no GPU): every option rejects
values outside its documented range with TN_EINVAL and keeps working after."""
import pytest

import paper_1908_08553_amd as tn

lib = tn.lib

# option: (accepted values, rejected values), as include/tn.h documents them
RANGES = {
    tn.TN_OPT_KERNEL_IMPL: ([0, 1], [-1, 2]),
    tn.TN_OPT_BATCH_THREADS: ([256, 512, 1024], [0, 128, 2048]),
    tn.TN_OPT_FUSE_STEPS: ([0, 1, 2], [-1, 3]),
    tn.TN_OPT_CHUNK_SCHEDULE: ([0, 1, 2], [-1, 3]),
    tn.TN_OPT_QUADRANT_STREAMS: ([0, 1], [-1, 2]),
    tn.TN_OPT_CHAIN_STEPS: ([0, 1], [-1, 2]),
    tn.TN_OPT_RING_OPERAND_SCALE: ([0, 1], [-1, 2]),
    tn.TN_OPT_CHUNK_STREAM: ([0, 1, 2, 65536], [-1, 65537]),
}
DEFAULTS = {tn.TN_OPT_KERNEL_IMPL: 0, tn.TN_OPT_BATCH_THREADS: 512, tn.TN_OPT_FUSE_STEPS: 2,
            tn.TN_OPT_CHUNK_SCHEDULE: 0, tn.TN_OPT_QUADRANT_STREAMS: 0,
            tn.TN_OPT_CHAIN_STEPS: 1, tn.TN_OPT_RING_OPERAND_SCALE: 0,
            tn.TN_OPT_CHUNK_STREAM: 1}


@pytest.mark.parametrize("opt", sorted(RANGES))
def test_option_ranges(opt):
    good, bad = RANGES[opt]
    try:
        for v in bad:
            assert lib.tn_set_option(opt, v) == tn.TN_EINVAL, (opt, v)
        for v in good:
            assert lib.tn_set_option(opt, v) == tn.TN_OK, (opt, v)
    finally:
        assert lib.tn_set_option(opt, DEFAULTS[opt]) == tn.TN_OK


def test_unknown_option():
    assert lib.tn_set_option(99, 0) == tn.TN_EINVAL
