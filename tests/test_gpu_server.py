"""GPU serving path: many streams batched into the same launches.

A stream's result must not depend on the streams it shares launches with:
each stream tracked inside a mix of streams (different meshes, cameras and
arrival times, so that their frames are at different iterations in the same
launch) must end bit-identical to the same stream tracked by a single-stream
context and by a server holding it alone.  Admission under a memory budget
queues streams instead of failing them; a rejected frame keeps the stream's
state.
"""
import sys

import numpy as np
import pytest

import synth

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


def _frames(body, th, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for f in range(n):
        t = th + np.where(body.angular, 0.01 * f, 0.002 * f)
        out.append(synth.render_frame(body.model, body.camera, synth.pose_surface(body.model, t), rng, 0.2, 0.002))
    return out


@pytest.fixture(scope="module")
def streams(tiny, small_body):
    """(model, camera, theta0, frames, submit step) per stream."""
    ragged_cam = dict(width=100, height=75, fx=90.0, fy=90.0, cx=49.5, cy=37.0)
    ragged = synth.make_body(3001, ragged_cam, 2.6)
    out = []
    for k, (body, start) in enumerate(((tiny.body, 0), (small_body, 0), (ragged, 2), (tiny.body, 7))):
        P = len(body.model["joint_parent"])
        rng = np.random.default_rng(40 + k)
        th = np.where(body.angular, rng.uniform(-0.05, 0.05, P), rng.uniform(-0.01, 0.01, P))
        frames = _frames(body, th, 3 if k != 1 else 2, 50 + k)
        th0 = th + np.where(body.angular, 0.02, 0.005)
        out.append((body.model, body.camera, th0, frames, start))
    return out


def _params():
    return dict(synth.default_params(1, 5, 0.05, lambda_k=0.1), active=None)


def _run_server(T, streams, which, budget=1 << 36, close_done=False):
    sv = T.track_server_create(_params(), budget, 64)
    try:
        ids, pending = {}, {}
        step = 0
        results = {}
        done = {k: 0 for k in which}
        order = []
        while True:
            for k in which:
                m, cam, th0, frames, start = streams[k]
                if step == start:
                    ids[k] = T.track_server_open(sv, m, cam, th0)
                    for f, d in enumerate(frames):
                        T.track_server_submit(sv, ids[k], d, tag=100 * k + f)
            if all(done[k] == len(streams[k][3]) for k in which) and step > max(streams[k][4] for k in which):
                break
            T.track_server_step(sv)
            for c in T.track_server_poll(sv):
                k = c["tag"] // 100
                assert c["status"] == 0, c
                assert c["stream"] == ids[k]
                assert c["tag"] % 100 == done[k], "frames of a stream complete in order"
                done[k] += 1
                order.append(k)
                if done[k] == len(streams[k][3]):
                    P, V = len(streams[k][0]["joint_parent"]), streams[k][0]["rest_xyz"].shape[0]
                    results[k] = T.track_server_state(sv, ids[k], P, V)
                    if close_done:
                        T.track_server_close(sv, ids[k])
            step += 1
            assert step < 500
        return results, order
    finally:
        T.track_server_destroy(sv)


def _run_alone(T, stream):
    m, cam, th0, frames, _ = stream
    trk = T.Tracker(m, cam, _params(), th0)
    try:
        for d in frames:
            assert trk.frame(d) == 0, T.track_last_error()
        th, phi, _, _ = trk.state(want_verts=False)
        return th, phi
    finally:
        trk.close()


def test_mix_equals_alone_bit_for_bit(T, streams):
    _say("[server] mix of 4 streams vs single-stream contexts and servers holding one stream")
    mix, order = _run_server(T, streams, [0, 1, 2, 3])
    _say(f"  completion order {order}")
    assert len(set(order[:3])) > 1, "streams interleave"
    for k in range(4):
        th_a, phi_a = _run_alone(T, streams[k])
        th_s, phi_s = _run_server(T, streams, [k])[0][k]
        th_m, phi_m = mix[k]
        assert np.array_equal(th_m, th_a) and np.array_equal(phi_m, phi_a), k
        assert np.array_equal(th_m, th_s) and np.array_equal(phi_m, phi_s), k


def test_admission_queues_under_a_budget(T, streams):
    _say("[server] admission under a budget of two streams")
    probe = T.track_server_create(_params(), 1 << 36, 64)
    try:
        sizes = []
        for k in (0, 1, 2):
            m, cam, th0, _, _ = streams[k]
            before = T.track_server_info(probe)["bytes_used"]
            T.track_server_open(probe, m, cam, th0)
            sizes.append(T.track_server_info(probe)["bytes_used"] - before)
    finally:
        T.track_server_destroy(probe)
    budget = sizes[0] + sizes[1] + sizes[2] // 2
    sv = T.track_server_create(_params(), budget, 64)
    try:
        ids = []
        for k in (0, 1, 2):
            m, cam, th0, frames, _ = streams[k]
            ids.append(T.track_server_open(sv, m, cam, th0))
            for f, d in enumerate(frames):
                T.track_server_submit(sv, ids[-1], d, tag=100 * k + f)
        info = T.track_server_info(sv)
        _say(f"  sizes {sizes} budget {budget} -> {info}")
        assert info["resident"] == 2 and info["waiting"] == 1 and info["bytes_used"] <= budget
        done = {0: 0, 1: 0, 2: 0}
        for _ in range(400):
            if all(done[k] == len(streams[k][3]) for k in done):
                break
            T.track_server_step(sv)
            for c in T.track_server_poll(sv):
                k = c["tag"] // 100
                assert c["status"] == 0
                done[k] += 1
                if done[k] == len(streams[k][3]) and k != 2:
                    if k == 0:
                        th_q, phi_q = T.track_server_state(sv, ids[0], len(streams[0][0]["joint_parent"]),
                                                           streams[0][0]["rest_xyz"].shape[0])
                    T.track_server_close(sv, ids[k])
        assert all(done[k] == len(streams[k][3]) for k in done), done
        P, V = len(streams[2][0]["joint_parent"]), streams[2][0]["rest_xyz"].shape[0]
        th2, phi2 = T.track_server_state(sv, ids[2], P, V)
    finally:
        T.track_server_destroy(sv)
    th_a, phi_a = _run_alone(T, streams[2])
    assert np.array_equal(th2, th_a) and np.array_equal(phi2, phi_a)
    th_a0, phi_a0 = _run_alone(T, streams[0])
    assert np.array_equal(th_q, th_a0) and np.array_equal(phi_q, phi_a0)


def test_a_stream_alone_exceeding_the_budget_is_refused(T, streams):
    sv = T.track_server_create(_params(), 1 << 20, 4)
    try:
        m, cam, th0, _, _ = streams[1]
        with pytest.raises(T.TrackError) as e:
            T.track_server_open(sv, m, cam, th0)
        assert e.value.code == T.TRACK_E_BUDGET
    finally:
        T.track_server_destroy(sv)


def test_rejected_frame_keeps_the_stream_state(T, streams):
    _say("[server] empty frame in the middle of a stream")
    m, cam, th0, frames, _ = streams[1]
    P, V = len(m["joint_parent"]), m["rest_xyz"].shape[0]
    sv = T.track_server_create(_params(), 1 << 36, 8)
    try:
        sid = T.track_server_open(sv, m, cam, th0)
        T.track_server_submit(sv, sid, frames[0], tag=0)
        T.track_server_submit(sv, sid, np.zeros_like(frames[0]), tag=1)
        T.track_server_submit(sv, sid, frames[1], tag=2)
        got = []
        for _ in range(100):
            T.track_server_step(sv)
            got += T.track_server_poll(sv)
            if len(got) == 1 and "after0" not in locals():
                after0 = T.track_server_state(sv, sid, P, V)
            if len(got) == 2 and "after1" not in locals():
                after1 = T.track_server_state(sv, sid, P, V)
            if len(got) == 3:
                break
        assert [c["status"] for c in got] == [0, T.TRACK_E_LOST, 0]
        assert np.array_equal(after0[0], after1[0]) and np.array_equal(after0[1], after1[1])
        th_s, phi_s = T.track_server_state(sv, sid, P, V)
    finally:
        T.track_server_destroy(sv)
    # the same frames without the empty one, tracked alone
    th_a, phi_a = _run_alone(T, (m, cam, th0, [frames[0], frames[1]], 0))
    assert np.array_equal(th_s, th_a) and np.array_equal(phi_s, phi_a)


def test_served_stream_matches_the_oracle_iteration_by_iteration(T, streams):
    """One stream served inside a mix (three other streams with frames in
    flight at different iterations) against the float64 oracle: the server
    runs one Gauss-Newton iteration per frame here, and each iteration of
    the checked stream starts from the oracle's state (the stream is opened
    with it), so every served result is compared with the oracle's step
    from the same state.  Bar: 1e-4 rad per joint angle, 1e-4 m per root
    translation and per vertex (both surfaces skinned by the oracle in
    float64)."""
    import oracle

    _say("[server] served stream vs oracle, iteration by iteration, inside a mix")
    one = dict(synth.default_params(1, 1, 0.05, lambda_k=0.1), active=None)
    m, cam, th0, frames, _ = streams[1]
    P, V = len(m["joint_parent"]), m["rest_xyz"].shape[0]
    body_ang = np.array([t == 0 for t in m["joint_type"]])
    sv = T.track_server_create(one, 1 << 36, 64)
    worst = [0.0, 0.0, 0.0]
    try:
        for k in (0, 2, 3):   # background traffic
            mb, cb, tb, fb, _ = streams[k]
            sid = T.track_server_open(sv, mb, cb, tb)
            for rep in range(40):
                T.track_server_submit(sv, sid, fb[rep % len(fb)], tag=1000 * k + rep)
        for _ in range(3):
            T.track_server_step(sv)
        th, phi = th0.copy(), np.zeros((V, 3))
        for f, depth in enumerate(frames):
            for it in range(5):
                sid = T.track_server_open(sv, m, cam, th, phi.astype(np.float32))
                T.track_server_submit(sv, sid, depth, tag=7)
                res = None
                for _ in range(200):
                    T.track_server_step(sv)
                    for c in T.track_server_poll(sv):
                        if c["tag"] == 7:
                            assert c["status"] == 0, c
                            res = T.track_server_state(sv, sid, P, V)
                    if res is not None:
                        break
                assert res is not None
                assert T.track_server_info(sv)["frames_in_progress"] > 0, "the mix is still running"
                T.track_server_close(sv, sid)
                th_o, phi_o = th.copy(), phi.astype(np.float32).astype(np.float64)
                oracle.track_frame(m, cam, one, th_o, phi_o, phi_o.copy(), depth=depth)
                vg, _ = oracle.skin(m, res[0], res[1].astype(np.float64))
                vo, _ = oracle.skin(m, th_o, phi_o)
                d = np.abs(res[0] - th_o)
                e = (d[body_ang].max(), d[~body_ang].max(), np.abs(vg - vo).max())
                worst = [max(a, b) for a, b in zip(worst, e)]
                _say(f"  frame {f} it {it}: joint {e[0]:.1e} rad, root {e[1]:.1e} m, vertex {e[2]:.1e} m")
                th, phi = th_o, phi_o
    finally:
        T.track_server_destroy(sv)
    assert worst[0] <= 1e-4 and worst[1] <= 1e-4 and worst[2] <= 1e-4, worst
