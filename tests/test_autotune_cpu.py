"""Host-side checks of the autotuner (no GPU): every choice is admissible for
its product (schedule supports the shape and beta, temporaries within the
memory budget, digit base only where its bounds hold), overwriting schedules
are never chosen automatically, fixed inputs are respected, and the cache file
round-trips between processes.  Also the benchmark's refusal of more than one
GPU."""
import json
import os
import subprocess
import sys

import pytest

from paper_0707_2347_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(capi.LIB_PATH),
                                reason="libwsmul.so not built")

SHAPES = [(64, 64, 64), (333, 444, 555), (1024, 512, 768), (4096, 4096, 4096),
          (8192, 4096, 8192), (2000, 3000, 100), (16384, 16384, 16384), (1, 70000, 1)]
PRIMES = [3, 65521, 1048573, 8388593, 16777213]


def _choice(m, k, n, p, beta=0, budget=(1 << 64) - 1, schedule=capi.WS_AUTO, levels=-1,
            base=capi.WS_BASE_AUTO, blocks=0):
    return capi.wsmul_autotune(m, k, n, p, capi.WS_F64, budget, schedule, levels, base, beta,
                               blocks)[:4]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("beta", [0, 7])
def test_choice_is_admissible(shape, p, beta):
    m, k, n = shape
    st, sched, lev, base = _choice(m, k, n, p, beta)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert sched in (capi.WS_CLASSICAL, capi.WS_TWO_TEMP, capi.WS_READONLY_INPLACE,
                     capi.WS_HL_THREE_TEMP)
    assert base in (capi.WS_BASE_F64_MFMA, capi.WS_BASE_I8_LIMBS)
    if sched == capi.WS_CLASSICAL:
        assert lev == 0
    else:
        assert lev >= 1 and min(m, k, n) >> lev >= 32
    if beta:
        assert sched != capi.WS_READONLY_INPLACE          # Algorithm 2 computes C = A*B only
    if base == capi.WS_BASE_I8_LIMBS:
        assert p <= 16711423 and k <= 32768
    # the chosen plan exists and its temporaries are what the library reports
    nbytes = capi.wsmul_workspace_bytes(m, k, n, capi.WS_F64, sched, lev, int(beta != 0))
    assert nbytes >= 0


@pytest.mark.parametrize("shape,p", [((4096, 4096, 4096), 65521), ((8192, 4096, 8192), 8388593),
                                     ((1024, 1024, 1024), 1048573)])
def test_budget_is_respected(shape, p):
    m, k, n = shape
    for budget in (0, 1 << 20, 64 << 20, 1 << 30):
        st, sched, lev, base = _choice(m, k, n, p, 0, budget)
        assert st == capi.WS_OK, capi.wsmul_last_error()
        assert capi.wsmul_workspace_bytes(m, k, n, capi.WS_F64, sched, lev, 0) <= budget
    # with no room at all an accumulating product still has the classical product
    st, sched, lev, base = _choice(m, k, n, p, 3, 0)
    assert st == capi.WS_OK and sched == capi.WS_CLASSICAL


def test_fixed_inputs_are_kept():
    st, sched, lev, base = _choice(2048, 2048, 2048, 65521, 0, schedule=capi.WS_TWO_TEMP, levels=2,
                                   base=capi.WS_BASE_F64_MFMA)
    assert (st, sched, lev, base) == (capi.WS_OK, capi.WS_TWO_TEMP, 2, capi.WS_BASE_F64_MFMA)
    st, sched, lev, base = _choice(2048, 2048, 2048, 65521, 0, schedule=capi.WS_READONLY_INPLACE)
    assert st == capi.WS_OK and sched == capi.WS_READONLY_INPLACE and lev >= 1
    st, sched, lev, base = _choice(2048, 2048, 2048, 65521, 0, base=capi.WS_BASE_F64_MFMA)
    assert st == capi.WS_OK and base == capi.WS_BASE_F64_MFMA


@pytest.mark.parametrize("n,p,budget", [(16384, 8388593, 512 << 20), (8192, 1048573, 100 << 20)])
def test_blocked_accumulation_under_small_budget(n, p, budget):
    """An accumulating product whose unblocked schedules do not fit the budget
    (Table 9 needs 2(n/2)^2 entries at one level) still gets a Winograd plan:
    Section 7.2's blocks, with temporaries within the budget."""
    assert capi.wsmul_workspace_bytes(n, n, n, capi.WS_F64, capi.WS_TWO_TEMP, 1, 1) > budget
    st, sched, lev, base, t = capi.wsmul_autotune(n, n, n, p, capi.WS_F64, budget, capi.WS_AUTO,
                                                  -1, capi.WS_BASE_F64_MFMA, 3)
    assert st == capi.WS_OK, capi.wsmul_last_error()
    assert sched in (capi.WS_BLOCKED, capi.WS_BLOCKED_ACC) and lev >= 1 and 2 <= t <= 4
    info = capi.wsmul_plan_info(capi.make_args(n, n, n, p, beta=3, schedule=sched, levels=lev,
                                               blocks=t))
    assert info.workspace_bytes <= budget
    # a fixed blocked schedule keeps the caller's t
    st, sched2, lev2, _, t2 = capi.wsmul_autotune(n, n, n, p, capi.WS_F64, budget,
                                                  capi.WS_BLOCKED_ACC, -1,
                                                  capi.WS_BASE_F64_MFMA, 3, 4)
    assert st == capi.WS_OK and sched2 == capi.WS_BLOCKED_ACC and t2 == 4 and lev2 >= 1


def test_overwriting_schedules_never_chosen():
    for shape in SHAPES:
        for beta in (0, 1):
            st, sched, _, _ = _choice(*shape, 65521, beta)
            assert sched not in (capi.WS_OVERWRITE, capi.WS_OVR, capi.WS_ACCR)


def test_degenerate_shapes():
    for shape in [(0, 5, 5), (5, 0, 5), (5, 5, 0)]:
        st, sched, lev, base = _choice(*shape, 65521)
        assert (st, sched, lev) == (capi.WS_OK, capi.WS_CLASSICAL, 0)


def test_bad_arguments():
    assert _choice(64, 64, 64, 1)[0] == capi.WS_EINVAL
    assert _choice(64, 64, 64, 1 << 24)[0] == capi.WS_EINVAL
    assert _choice(-1, 64, 64, 65521)[0] == capi.WS_EINVAL
    assert _choice(64, 64, 64, 65521, schedule=99)[0] == capi.WS_ESCHEDULE


def test_fixed_schedule_errors_are_the_schedules_own():
    """With the schedule fixed, a request the schedule cannot take fails with
    that schedule's status, not with a memory-budget error."""
    assert _choice(64, 64, 64, 65521, beta=1, schedule=capi.WS_READONLY_INPLACE,
                   levels=1)[0] == capi.WS_ESCHEDULE
    assert _choice(64, 64, 48, 65521, schedule=capi.WS_OVL)[0] == capi.WS_ESHAPE
    st, sched, lev, _ = _choice(48, 48, 48, 65521, schedule=capi.WS_OVL)
    assert (st, sched) == (capi.WS_OK, capi.WS_OVL) and lev >= 1
    assert _choice(4096, 4096, 4096, 65521, beta=1, budget=1000, schedule=capi.WS_TWO_TEMP,
                   levels=3)[0] == capi.WS_ENOMEM


def test_cache_file_round_trip(tmp_path):
    """A fresh process writes its choices to WSMUL_TUNE_CACHE; a second one
    reads them back (the file holds one JSON object per line)."""
    cache = tmp_path / "tune.jsonl"
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_0707_2347_amd import capi\n"
            "print(capi.wsmul_autotune(3000, 2000, 1000, 1048573)[1:4])\n" % ROOT)
    env = dict(os.environ, WSMUL_TUNE_CACHE=str(cache))
    first = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=120)
    assert first.returncode == 0, first.stderr
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert (rec["m"], rec["k"], rec["n"], rec["p"]) == (3000, 2000, 1000, 1048573)
    assert str((rec["schedule"], rec["levels"], rec["base"])) == first.stdout.strip()
    # a planted entry is what the next process returns, so the file is read
    rec["schedule"], rec["levels"], rec["base"] = capi.WS_TWO_TEMP, 1, capi.WS_BASE_F64_MFMA
    cache.write_text(json.dumps(rec) + "\n")
    second = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                            text=True, timeout=120)
    assert second.returncode == 0, second.stderr
    assert second.stdout.strip() == str((capi.WS_TWO_TEMP, 1, capi.WS_BASE_F64_MFMA))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_digit_base_choices_at_16384():
    """The choices the measurements support at 16384^3 (same-box pairs in the
    design record): Table 1 at one level on the 8-bit digit base for C = AB mod
    1048573 (temporaries and inputs held as digit planes, 2-7% ahead of the
    classical digit product), the classical digit product for C <- AB + C (a
    tie with Table 2, decided for the schedule without temporaries), and the
    classical product with two digits mod 65521 (where a level loses)."""
    st, sched, lev, base, _ = capi.wsmul_autotune(16384, 16384, 16384, 1048573)
    assert st == capi.WS_OK and (sched, lev, base) == (capi.WS_TWO_TEMP, 1,
                                                        capi.WS_BASE_I8_LIMBS)
    st, sched, lev, base, _ = capi.wsmul_autotune(16384, 16384, 16384, 1048573, beta=3)
    assert st == capi.WS_OK and (sched, base) == (capi.WS_CLASSICAL, capi.WS_BASE_I8_LIMBS)
    st, sched, lev, base, _ = capi.wsmul_autotune(16384, 16384, 16384, 65521)
    assert st == capi.WS_OK and (sched, base) == (capi.WS_CLASSICAL, capi.WS_BASE_I8_LIMBS)
    # binary64 only: Winograd pays there (Table 1 with two or more levels)
    st, sched, lev, base, _ = capi.wsmul_autotune(16384, 16384, 16384, 1048573,
                                                 base=capi.WS_BASE_F64_MFMA)
    assert st == capi.WS_OK and sched == capi.WS_TWO_TEMP and lev >= 2
