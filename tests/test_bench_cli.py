"""bench.py's command-line contract that needs no GPU."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_help_lists_the_modes():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert p.returncode == 0
    for mode in ("throughput", "copy", "solve", "sweep", "warmstart", "paper", "network"):
        assert mode in p.stdout


def test_network_flop_count():
    # the U-Net's convolutions at 64^3: level-0 layers carry sum C_in*C_out =
    # 8*16 + 16*16 + 32*16 + 16*16 + 16*16, level 1 (32^3) 16*32 + 32*32 +
    # 64*32 + 32*32, level 2 (16^3) 32*64 + 64*64 + 128*64 + 64*64, level 3
    # (8^3) 64*128 + 128*128; each voxel-channel pair costs 2 * 27 FLOPs
    import types

    from paper_1503_08718_amd import warmstart as ws

    cc = [(64 ** 3, 1408), (32 ** 3, 4608), (16 ** 3, 18432), (8 ** 3, 24576)]
    fwd = 54.0 * sum(v * c for v, c in cc)
    assert ws.forward_flops(types.SimpleNamespace(batch=1, n=64)) == fwd
    assert ws.forward_flops(types.SimpleNamespace(batch=4, n=64)) == 4 * fwd
    # training: forward + weight gradient everywhere, input gradient except the first layer
    first = 54.0 * 64 ** 3 * 8 * 16
    assert ws.iteration_flops(types.SimpleNamespace(batch=1, n=64)) == 3 * fwd - first
