"""The exchange of the cooperative sweep (spread walkers), as a CPU model with
threads for workgroups (tests/spread_protocol_model.cc): sequence-tagged
mailbox words under relaxed atomics, partial sums added in slice order, and
the next move's atom position published by the worker that holds it.  Every
worker takes the decisions of a sequential run of the same arithmetic,
bitwise, and the final positions match it; a worker that stops publishing
makes the others give up within their poll limit, and every worker leaves."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("spread") / "spread_protocol_model")
    subprocess.run(["g++", "-std=c++17", "-O2", "-pthread", os.path.join(HERE, "spread_protocol_model.cc"),
                    "-o", exe], check=True)
    return exe


def run(exe, *args):
    out = subprocess.run([exe, *map(str, args)], check=True, capture_output=True, text=True, timeout=120)
    return out.stdout.split()


@pytest.mark.parametrize("C,n", [(2, 40), (3, 61), (8, 200), (14, 97)])
def test_all_workers_take_the_sequential_decisions(model, C, n):
    r = run(model, C, n, 20000, 1 << 30, -1)
    assert r[0] == "ok" and int(r[1]) == 20000
    assert 2000 < int(r[2]) < 18000   # both outcomes occur


@pytest.mark.parametrize("C,stall", [(2, 0), (2, 500), (4, 123)])
def test_a_stalled_worker_makes_the_others_give_up(model, C, stall):
    r = run(model, C, 64, 2000, 20000, stall)
    assert r[0] == "gaveup" and int(r[1]) == stall and int(r[2]) == C
