"""The benchmark's command-line contract on the host (no GPU needed): it measures one GPU and says so
when asked for more, and a counter figure is only reported for the kernel source and launch plan it
was taken on."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_needs_matching_plan_and_source():
    b = _bench()
    (kname, prec), ent = next(iter(b.TRAFFIC.items()))
    plan = dict(ent["plan"], nsplit_b=0, nsplit_y=0, x_variant=0, y_variant=0, pchunk=ent["plan"]["pchunk"])
    plan.update(ent["plan"])
    src_ok = all(b._sha(os.path.join(b.KSRC, f)) == h for f, h in ent["sha256"].items())
    assert b.traffic(kname, prec, plan) == (ent["bytes"] if src_ok else None)
    other = dict(plan, pchunk=plan["pchunk"] + 1)
    assert b.traffic(kname, prec, other) is None
    assert b.traffic("no_such_kernel", prec, plan) is None
