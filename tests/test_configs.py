"""The configuration files (paper_2602_14667_amd/configs/c1..c5.json): each
names a bench workload, every key of its 'bench' block is a flag of bench.py,
and bench.py accepts it (driven here with --gpus 2, which it refuses before
touching a GPU, so the check runs on the CPU).  A key that is not a flag is
rejected."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CFG = os.path.join(ROOT, "paper_2602_14667_amd", "configs")
NAMES = ["c1", "c2", "c3", "c4", "c5"]


def _bench(*argv):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


@pytest.mark.parametrize("name", NAMES)
def test_config_is_accepted(name):
    with open(os.path.join(CFG, f"{name}.json")) as fh:
        cfg = json.load(fh)
    assert cfg["name"] == name and cfg["description"]
    assert cfg["bench"]["workload"] in ("ot64", "hartmann", "turbulence", "batch", "closure")
    assert all(k.startswith("RRMHD_") for k in cfg.get("env", {}))
    r = _bench("--config", name, "--gpus", "2")
    assert r.returncode == 2 and "one GPU only" in r.stderr, r.stderr


def test_config_with_an_unknown_key_is_rejected(tmp_path):
    bad = tmp_path / "bad.json"
    bad.write_text(json.dumps({"name": "bad", "bench": {"workload": "turbulence",
                                                        "tile": "64x4"}}))
    r = _bench("--config", str(bad), "--gpus", "2")
    assert r.returncode == 2 and "unknown keys ['tile']" in r.stderr, r.stderr
