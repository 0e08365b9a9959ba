"""The agreement protocol of the cooperative sweep (spread walkers), as a CPU
model with threads for workgroups (tests/spread_protocol_model.cc): all
workers agree on every move's total, bitwise, in slice order; a worker that
stops arriving makes the others give up within their poll limit, and every
worker leaves (the GPU kernel follows the same steps, with the device's
atomics and fences)."""
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


@pytest.mark.parametrize("C", [2, 3, 8])
def test_all_workers_agree_on_every_move(model, C):
    assert run(model, C, 20000, 1 << 30, -1) == ["ok", "20000"]


@pytest.mark.parametrize("C,stall", [(2, 0), (2, 500), (4, 123)])
def test_a_stalled_worker_makes_the_others_give_up(model, C, stall):
    r = run(model, C, 2000, 20000, stall)
    assert r[0] == "gaveup" and int(r[1]) == stall and int(r[2]) == C
