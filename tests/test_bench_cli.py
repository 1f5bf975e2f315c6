"""The benchmark's command line on the host: more than one GPU is refused
with a message before anything touches a device, and every workload name
the help lists is accepted by the parser."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, 'bench.py'), '--gpus', '2'], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert 'one GPU only' in r.stderr
    assert r.stdout == ''


def test_workload_names_in_the_help():
    import importlib.util
    spec = importlib.util.spec_from_file_location('bench_mod', os.path.join(ROOT, 'bench.py'))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    doc = mod.__doc__
    for name in mod.WORKLOADS:
        assert name in doc, name
