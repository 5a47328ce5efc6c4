"""The fix-up protocol (Signal/Wait on ready flags, partial tiles in
per-workgroup slots, flags cleared by their reader for the next launch) run
by CPU threads under ThreadSanitizer, on schedules the planner produces.

tests/emu/fixup_emu.cpp emulates one workgroup per thread with release
stores and acquire loads on the flags and plain memory for the slots, so
ThreadSanitizer reports any slot read the protocol does not order after its
write.  Checked here: exact integer results over several launches that reuse
the slots and flags (owner fix-up and split fix-up), no race report, no flag
left raised; a dropped Signal ends in the bounded wait's timeout instead of a
hang; and, as a planted mistake, owners that skip the wait are reported."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emu", "fixup_emu.cpp")


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("emu") / "fixup_emu")
    res = subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=thread", "-pthread", SRC, "-o", out],
                         capture_output=True, text=True)
    if res.returncode != 0:
        pytest.skip(f"ThreadSanitizer build unavailable: {res.stderr[-300:]}")
    return out


def _plan(**kw):
    from paper_2212_08964_amd import skgemm as sk
    return sk.Plan(ta=sk.BF16, num_cus=64, occupancy=2, **kw)


def _run(emu, plan, launches=3, spin=200000, drop=-1, skip=0, units=4):
    info = plan.info()
    recs = plan.schedule()
    lines = [f"{info['grid']} {info['coop_s']} {units} {launches} {spin} {drop} {skip}"]
    lines += [" ".join(str(int(v)) for v in r) for r in recs]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=0 exitcode=66")
    return subprocess.run([emu], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=300,
                          env=env)


CASES = [
    # (shape, policy, forced grid, fixup)
    ((384, 384, 1024), "sk", 0, "owner"),          # basic Stream-K, model grid, owners with several peers
    ((384, 384, 1024), "sk", 36, "auto"),          # aligned split: split fix-up over 4 shares
    ((896, 384, 128), "2tile_sk_dp", 0, "owner"),  # two-tile hybrid
    ((2000, 1500, 333), "dp_1tile_sk", 0, "owner"),
    ((1000, 700, 900), "sk", 48, "auto"),          # split fix-up, 3 shares per tile
    ((1000, 700, 900), "sk", 77, "owner"),         # unaligned grid
    ((300, 500, 2048), "sk", 0, "auto"),
]


@pytest.mark.parametrize("shape,policy,g,fixup", CASES)
def test_protocol_exact_and_race_free(emu, shape, policy, g, fixup):
    M, N, K = shape
    p = _plan(M=M, N=N, K=K, policy=policy, force_g=g, fixup=fixup)
    assert p.info()["g_sk"] > 0
    res = _run(emu, p)
    assert "ThreadSanitizer" not in res.stderr, res.stderr[-2000:]
    assert res.returncode == 0, (res.stdout, res.stderr[-2000:])
    assert res.stdout.startswith("ok 3 launches")


@pytest.mark.parametrize("fixup", ["owner", "auto"])
def test_dropped_signal_times_out(emu, fixup):
    """A peer that never raises its flag: the waiting workgroup gives up after
    its spin limit and reports the timeout; every thread exits."""
    p = _plan(M=1000, N=700, K=900, policy="sk", force_g=77 if fixup == "owner" else 0, fixup=fixup,
              tile=(256, 256, 64))
    assert (p.info()["coop_s"] > 0) == (fixup == "auto")
    recs = p.schedule()
    partial_wg = next(r[0] for r in recs if r[5] == 1)
    res = _run(emu, p, launches=1, spin=2000, drop=partial_wg)
    assert res.returncode == 3, (res.stdout, res.stderr[-1000:])
    assert "timed out" in res.stdout


def test_planted_missing_wait_is_reported(emu):
    """Owners that read the peers' slots without waiting for their flags: the
    race on the slots is reported (or the sums come out wrong)."""
    p = _plan(M=384, N=384, K=1024, policy="sk", force_g=0, fixup="owner")
    res = _run(emu, p, launches=2, skip=1)
    assert "ThreadSanitizer: data race" in res.stderr or res.returncode == 1
