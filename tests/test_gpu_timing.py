"""Kernel timing through the C ABI: per-pass event timers inside frames and
the back-to-back repeat used for the benchmark's roofline figure.  Timing
must not change what a frame computes, and a reset after a repeat must give
the same frames as a fresh tracker."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_1711_07999_amd import track
    track.lib()
    return track


def test_timers_and_repeats(T, tiny):
    import torch

    _say("[timing] tiny arm, 3 frames")
    m, cam = tiny.body.model, tiny.body.camera
    frames = [torch.from_numpy(f).to("cuda:0") for f in tiny.frames[:3]]
    ref = T.Tracker(m, cam, tiny.params, tiny.theta0)
    trk = T.Tracker(m, cam, tiny.params, tiny.theta0)
    try:
        for k in range(len(T.KERNEL_NAMES)):
            T.track_kernel_timing(trk.ctx, k, True)
        for f in frames:
            assert ref.frame(f) == 0, T.track_last_error()
            assert trk.frame(f) == 0, T.track_last_error()
        th_r = ref.state()[0]
        th_t = trk.state()[0]
        assert np.array_equal(th_r, th_t), "timing changed the result"
        for name in ("skin", "assoc", "normal_eq", "solve"):
            n, ms = T.track_kernel_time(trk.ctx, T.KERNEL_NAMES.index(name))
            _say(f"  {name}: {n} launches, {ms:.3f} ms")
            assert n > 0 and ms > 0.0, name
        # the bucket index has no launch of its own
        assert T.track_kernel_time(trk.ctx, T.KERNEL_NAMES.index("bucket"))[0] == 0
        for k in range(len(T.KERNEL_NAMES)):
            T.track_kernel_timing(trk.ctx, k, False)
        for name in ("skin", "assoc", "normal_eq", "solve"):
            ms = T.track_kernel_bench(trk.ctx, T.KERNEL_NAMES.index(name), frames[-1], 20)
            _say(f"  repeat {name}: {ms * 1e3:.1f} us per launch")
            assert 0.0 < ms < 100.0, name
        with pytest.raises(RuntimeError):
            T.track_kernel_bench(trk.ctx, T.KERNEL_NAMES.index("bucket"), frames[-1], 20)
        # the repeats consumed the state: a reset gives a fresh tracker's frames
        trk.reset(tiny.theta0)
        ref.reset(tiny.theta0)
        for f in frames:
            assert ref.frame(f) == 0 and trk.frame(f) == 0, T.track_last_error()
        assert np.array_equal(ref.state()[0], trk.state()[0])
        assert np.array_equal(ref.state()[1], trk.state()[1])
    finally:
        trk.close()
        ref.close()
