"""bench.py's command line, on the CPU: a run on more than one GPU is
refused with a message (the library measures one GPU), and --tile maps to
the library's tile flags (-1, the autotuner, and 0 leave the default)."""

import importlib.util
import os
import subprocess
import sys

import paper_2301_08357_amd as pm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_tile_option_maps_to_flags():
    spec = importlib.util.spec_from_file_location("bench_cli", BENCH)
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)

    class Args:
        tile = 0

    for tile, flag in ((-1, 0), (0, 0), (128, pm.PM_TILE_128), (256, pm.PM_TILE_256), (512, pm.PM_TILE_512)):
        Args.tile = tile
        assert bench.tile_flag_of(Args) == flag
