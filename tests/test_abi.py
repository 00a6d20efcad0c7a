"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function include/track.h declares, and rejects invalid input before
touching the device."""
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from paper_1711_07999_amd import track as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "track.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(track_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("track_init", "track_frame", "track_state"):
        assert must in names
    assert set(names) == set(T.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = T.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", T.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(track_\w+)", out))
    assert set(declared_functions()) <= exported


def _model():
    return synth.workload_tiny().body


@pytest.mark.parametrize("mutate,msg", [
    (lambda m, c, p: m.__setitem__("joint_parent", np.array([0] + list(m["joint_parent"][1:]), np.int32)), "parents"),
    (lambda m, c, p: m.__setitem__("faces", np.where(m["faces"] == 7, 10 ** 6, m["faces"]).astype(np.int32)), "face"),
    (lambda m, c, p: m.__setitem__("skin_w", (m["skin_w"] * 0.5).astype(np.float32)), "sum to 1"),
    (lambda m, c, p: m.__setitem__("joint_axis", (m["joint_axis"] * 2).astype(np.float32)), "unit"),
    (lambda m, c, p: c.__setitem__("fx", -1.0), "intrinsics"),
    (lambda m, c, p: p.__setitem__("tau", 0.0), "tau"),
    (lambda m, c, p: p.__setitem__("n_iters", 0), "n_iters"),
    (lambda m, c, p: m.__setitem__("scale", 0.0), "scale"),
    (lambda m, c, p: m.__setitem__("scale", float("nan")), "scale"),
])
def test_invalid_input_is_rejected(mutate, msg):
    body = _model()
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in body.model.items()}
    c = dict(body.camera)
    p = dict(synth.default_params(8, 2, 0.1))
    mutate(m, c, p)
    with pytest.raises(T.TrackError) as e:
        T.track_init(m, c, p, np.zeros(8))
    assert e.value.code == T.TRACK_E_INVALID
    assert msg in str(e.value)


def test_allocator_without_free_is_rejected():
    """A provider must give both calls; checked before any device work."""
    body = _model()
    half = T.track_allocator(T.ALLOC_FN(lambda n, u: None), T.FREE_FN(), None)
    with pytest.raises(T.TrackError) as e:
        T.track_init(body.model, body.camera, synth.default_params(8, 2, 0.1), np.zeros(8), allocator=half)
    assert e.value.code == T.TRACK_E_INVALID
    assert "allocator" in str(e.value)
