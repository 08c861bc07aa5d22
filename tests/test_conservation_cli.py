"""Host-side checks of the conservation study's argument handling (no GPU)."""

import pytest

from paper_1901_08532_amd import conservation


def test_single_precision_with_block_steps_is_refused_before_any_gpu_work():
    with pytest.raises(ValueError, match="single precision"):
        conservation.run(n=64, time_units=0.0625, precision="sp", mode="block")
    with pytest.raises(SystemExit) as e:
        conservation.main(["--mode", "block", "--precisions", "fp64,sp"])
    assert e.value.code == 2


def test_bad_mode_step_and_precision_are_refused():
    with pytest.raises(ValueError):
        conservation.run(n=64, mode="neither")
    with pytest.raises(ValueError, match="divide"):
        conservation.run(n=64, dt=0.1)
    with pytest.raises(SystemExit):
        conservation.main(["--precisions", "fp128"])


def test_precision_names_map_to_the_library_constants():
    from paper_1901_08532_amd import h6

    assert conservation.PRECISIONS == {"fp64": h6.H6_FP64, "mixed": h6.H6_MIXED,
                                       "ex": h6.H6_EX, "sp": h6.H6_SP}
    assert (h6.H6_FP64, h6.H6_MIXED, h6.H6_EX, h6.H6_SP) == (0, 1, 2, 3)
