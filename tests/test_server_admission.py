"""The fit server's admission policy and arena (csrc/admission.h, the code
the server runs) against a stub executor on the CPU: a byte budget, a mock
clock and requests that each run a given number of ticks.  This forces
refusal, queueing and retirement without a GPU."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def stub(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("stub") / "stub_admission")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-o", exe,
                           os.path.join(HERE, "stub_admission.cpp")])

    def run(lines):
        out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                             check=True, timeout=60).stdout.strip().splitlines()
        assert len(out) == len(lines)
        return out
    return run


def _stream(stub, arena, slots, per_fit, reqs):
    line = f"S {arena} {slots} {per_fit} {len(reqs)} " + " ".join(f"{f} {t}" for f, t in reqs)
    out = stub([line])[0]
    ticks, tail = out.split("|")
    v = [int(x) for x in ticks.split()]
    peak, empty, stalled = (int(x) for x in tail.split())
    return list(zip(v[0::2], v[1::2])), peak, empty, stalled


def test_memory_bounds_the_admitted_set(stub):
    # three 256,000-byte fits and the batch workspace of three (3 x 25,600)
    # fit a 1,024,000-byte arena; a fourth does not until one retires
    times, peak, empty, stalled = _stream(stub, 1_024_000, 4, 25_600,
                                          [(256_000, 3), (256_000, 2), (256_000, 4),
                                           (256_000, 1), (256_000, 1)])
    assert times == [(0, 3), (0, 2), (0, 4), (2, 3), (3, 4)]
    assert peak <= 1_024_000 and empty == 1 and stalled == 0


def test_first_come_first_served_no_overtaking(stub):
    # the big second request must wait for the first to retire, and the small
    # third one, although it would fit, is not admitted before it
    times, peak, empty, stalled = _stream(stub, 1_000_000, 8, 1_000,
                                          [(600_000, 5), (700_000, 2), (10_000, 1)])
    assert times[0] == (0, 5)
    assert times[1][0] == 5
    assert times[2][0] >= times[1][0]
    assert empty == 1 and stalled == 0


def test_slot_limit(stub):
    reqs = [(1_000, 3)] * 6
    times, peak, empty, stalled = _stream(stub, 10_000_000, 2, 256, reqs)
    for t in range(0, 12):
        running = sum(1 for a, d in times if a <= t < d)
        assert running <= 2
    assert [a for a, _ in times] == [0, 0, 3, 3, 6, 6]
    assert empty == 1


def test_request_that_never_fits_stalls_the_queue(stub):
    # a workspace larger than the arena is never admitted (the server
    # rejects such a request with NO_MEMORY when it is submitted)
    times, peak, empty, stalled = _stream(stub, 100_000, 4, 1_000, [(50_000, 2), (200_000, 1)])
    assert times[0] == (0, 2) and times[1] == (-1, -1)
    assert stalled == 1 and empty == 1


def test_arena_first_fit_and_coalescing(stub):
    out = stub(["A 4096 6  1024 1024 1024 -2 2048 -1",
                "A 4096 7  1024 1024 1024 -2 -1 2048 1024",
                "A 4096 5  100 300 -1 512 200"])
    # a 2,048-byte request fails on two separate 1,024-byte holes ...
    assert out[0] == "0 1024 2048 -1 | 1024"
    # ... and succeeds once the neighbouring holes merge
    assert out[1] == "0 1024 2048 0 3072 | 4096"
    # sizes round up to 256-byte units; the first hole that fits is taken:
    # 512 bytes skip the freed 256-byte hole, 200 bytes fill it
    assert out[2] == "0 256 768 0 | 1280"
