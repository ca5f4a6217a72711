"""GPU: the continuous-batching fit server.

Each request's result must be the same served in a mix of other requests as
run alone (bitwise: the histograms are exact integer sums and every selection
is per fit), and two of them are also checked against the FP64 oracle.
"""
import time

import numpy as np
import pytest

from paper_2110_03513_amd import cwb, datagen
from tests.parity import compare

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _requests():
    out = []
    variants = ["cwb", "acwb", "hcwb"]
    for i in range(8):
        rng = np.random.default_rng(7000 + i)
        n = int(rng.integers(8_000, 60_000))
        p = int(rng.integers(3, 25))
        v = variants[i % 3]
        loss = "l2" if i % 2 == 0 else "binomial"
        cat = 2 if i in (3, 5) else 0  # categorical learners: the LDS-copies kernel variant
        prob = datagen.additive_problem(n, p, seed=7000 + i, n_informative=min(3, p), loss=loss,
                                        n_bins=int(np.sqrt(n)), M=int(rng.integers(30, 160)),
                                        variant=v, gamma=0.05 if v == "acwb" else 0.2,
                                        patience=3, val_frac=0.2 if v == "hcwb" else 0.0,
                                        n_cat=cat, n_informative_cat=min(cat, 1))
        out.append(prob)
    return out


def _drain(srv, tickets, limit_s=120.0):
    done = {}
    t0 = time.time()
    while len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        assert time.time() - t0 < limit_s, "server did not finish in time"
        time.sleep(0.002)
    return done


@pytest.mark.parametrize("setup", ["host", "device"])
def test_server_alone_vs_mix(setup):
    """Alone with the host setup; in the server with the host setup, or
    with binning, counts and solves on the GPU during each upload."""
    probs = _requests()
    _say("8 requests alone")
    alone = [cwb.fit(dict(p, setup="host")) for p in probs]
    _say(f"8 requests through the server, staggered, setup={setup}")
    srv = cwb.Server(arena_bytes=1 << 30, max_slots=4, quantum=16)
    tickets = []
    for p in probs:
        tickets.append(srv.submit(dict(p, setup=setup)))
        time.sleep(0.01)
    done = _drain(srv, tickets)
    st = srv.stats()
    srv.close()
    _say(f"stats {st}")
    assert st["completed"] == 8 and st["rejected"] == 0
    assert st["arena_peak"] <= 1 << 30
    for t, a, p in zip(tickets, alone, probs):
        r = done[t]
        assert r["status"] == 0, r.get("error")
        np.testing.assert_array_equal(r["k"], a["k"])
        np.testing.assert_array_equal(r["f"], a["f"])
        assert r["f0"] == a["f0"]
    for i in (1, 2):  # an ACWB and an HCWB request against the oracle
        g = dict(alone[i])
        g["k"] = done[tickets[i]]["k"]
        g["f"] = done[tickets[i]]["f"]
        compare(g, probs[i])


def test_server_admission_under_a_small_arena():
    probs = _requests()[:6]
    sizes = [cwb.workspace_bytes(p) for p in probs]
    arena = int(2.2 * max(sizes)) + (8 << 20)
    _say(f"arena {arena} bytes for workspaces {sizes}")
    alone = [cwb.fit(p) for p in probs]
    srv = cwb.Server(arena_bytes=arena, max_slots=16, quantum=8)
    tickets = [srv.submit(p) for p in probs]
    # the uint16 index matrix alone (2 n p bytes) exceeds the arena
    big_n = arena // (2 * 40) + 1000
    big = datagen.additive_problem(big_n, 40, seed=99, n_informative=3, n_bins=600, M=10)
    t_big = srv.submit(big)
    done = _drain(srv, tickets + [t_big])
    st = srv.stats()
    srv.close()
    _say(f"stats {st}")
    assert done[t_big]["status"] == cwb.CWB_E_NO_MEMORY
    assert st["completed"] == 6 and st["rejected"] == 1
    assert st["arena_peak"] <= arena
    for t, a in zip(tickets, alone):
        np.testing.assert_array_equal(done[t]["k"], a["k"])
        np.testing.assert_array_equal(done[t]["f"], a["f"])


def test_server_reports_setup_errors_per_request():
    good = _requests()[0]
    bad = dict(good)
    bad["loss"] = "binomial"
    bad["y"] = np.full_like(good["y"], 2.0)  # binomial labels must be 0 or 1
    # a constant feature, found by the device setup pass during the upload
    const = dict(good, setup="device", x=good["x"].copy())
    const["x"][:, 1] = 0.5
    srv = cwb.Server(arena_bytes=256 << 20, max_slots=2, quantum=10)
    tb = srv.submit(bad)
    tc = srv.submit(const)
    tg = srv.submit(good)
    done = _drain(srv, [tb, tc, tg])
    srv.close()
    assert done[tb]["status"] == cwb.CWB_E_INVALID_ARG and "error" in done[tb]
    assert done[tc]["status"] == cwb.CWB_E_INVALID_ARG
    assert "constant feature 1" in done[tc]["error"]
    assert done[tg]["status"] == 0
    np.testing.assert_array_equal(done[tg]["k"], cwb.fit(good)["k"])


def test_server_close_with_requests_in_flight():
    """Closing while requests are queued, in setup, uploading or running:
    queued ones are cancelled, admitted ones finish, and close returns."""
    probs = _requests()
    srv = cwb.Server(arena_bytes=1 << 30, max_slots=3, quantum=5)
    for p in probs:
        srv.submit(p)
    t0 = time.time()
    while srv.stats()["in_flight"] < 1:  # at least one admitted (uploading or running)
        assert time.time() - t0 < 30.0, "no request was admitted"
        time.sleep(0.001)
    _say(f"closing with stats {srv.stats()}")
    t0 = time.time()
    srv.close()
    _say(f"close took {time.time() - t0:.2f} s")
    # a new server on the same device still works
    srv = cwb.Server(arena_bytes=256 << 20, max_slots=2, quantum=10)
    t = srv.submit(probs[0])
    done = _drain(srv, [t])
    srv.close()
    assert done[t]["status"] == 0
    np.testing.assert_array_equal(done[t]["k"], cwb.fit(probs[0])["k"])
