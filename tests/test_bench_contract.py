"""The JSON line bench.py prints: the fields and invariants a reader of the
benchmark relies on (one line; value, unit, steps and warmup as asked;
roofline frac = achieved / peak; the config names its workload), for the
apply, quadcoll, steady and RK4 lines.  The multi-GPU refusal runs on the
CPU; the rest needs a GPU and times a step or two of each workload."""
import json
import math
import sys

import pytest

sys.path.insert(0, __import__("os").path.dirname(__import__("os").path.dirname(__file__)))
import bench  # noqa: E402


def run_bench(monkeypatch, capsys, args):
    monkeypatch.setattr(sys, "argv", ["bench.py"] + args)
    bench.main()
    lines = [l for l in capsys.readouterr().out.splitlines() if l.strip()]
    assert len(lines) == 1, lines
    return json.loads(lines[0])


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    rec = json.loads(capsys.readouterr().out.strip())
    assert rec["n_gpus"] == 2 and "one GPU" in rec["error"]


def check_line(rec, steps, warmup):
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in rec, k
    assert rec["n_gpus"] == 1 and rec["steps"] == steps and rec["warmup"] == warmup
    assert rec["value"] > 0 and math.isfinite(rec["value"]) and rec["ms_per_step"] > 0
    assert isinstance(rec["higher_is_better"], bool) and rec["scaling"] in ("weak", "strong")
    assert isinstance(rec["config"], dict) and rec["config"].get("workload")
    r = rec["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["bound"] in ("hbm", "mfma", "alu") and r["unit"] in ("GB/s", "TFLOP/s")
    assert r["peak"] > 0 and r["achieved"] > 0
    assert abs(r["frac"] - r["achieved"] / r["peak"]) <= 1e-9 * r["frac"]
    assert r["traffic"] is None or r["traffic"] > 0


@pytest.mark.gpu
@pytest.mark.parametrize("args,steps,warmup", [
    (["--steps", "2", "--warmup", "1", "--no-cpu"], 2, 1),
    (["--op", "quadcoll", "--steps", "1", "--warmup", "1", "--no-cpu"], 1, 1),
    (["--op", "steady", "--steps", "1", "--warmup", "1", "--no-cpu"], 1, 1),
    # the RK4 line times the paper's fixed workload of 100 steps
    (["--op", "rk4", "--steps", "1", "--warmup", "1", "--no-cpu"], 100, 1),
])
def test_bench_line(monkeypatch, capsys, args, steps, warmup):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    rec = run_bench(monkeypatch, capsys, args)
    check_line(rec, steps, warmup)
    if "--op" not in args:
        # the headline apply line: the fused kernel's roofline, FP32 error against FP64 within the bar
        assert rec["roofline"]["kernel"].startswith("k_fused<32, ")
        assert rec["rel_err_vs_fp64"]["max"] <= 1e-5
        assert rec["vs_baseline"] is None
