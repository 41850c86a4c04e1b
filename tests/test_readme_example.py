"""The C example of the README, compiled against include/rcell.h and linked to the built library
with the command the README gives: it must keep matching the ABI.  Without a usable GPU it runs
up to rcell_create, which reports the device error through rcell_last_error and exits with 1."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_1902_09171_amd")


def _gpu_present():
    import torch
    return torch.cuda.device_count() > 0


def test_readme_c_example_builds_and_reports_errors(tmp_path):
    if not os.path.exists(os.path.join(LIB_DIR, "librcell.so")):
        pytest.skip("librcell.so is not built")
    text = open(os.path.join(ROOT, "README.md")).read()
    src = re.search(r"```c\n(.*?)```", text, re.S).group(1)
    c = tmp_path / "example.c"
    c.write_text(src)
    exe = tmp_path / "example"
    subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(c),
                           "-L", LIB_DIR, "-lrcell", "-Wl,-rpath-link,/opt/rocm/lib", "-o", str(exe)])
    if _gpu_present():
        return                                    # running it is the GPU's business
    env = dict(os.environ, LD_LIBRARY_PATH=f"{LIB_DIR}:/opt/rocm/lib")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 1
    assert r.stderr.startswith("create: ") and "hip" in r.stderr.lower(), r.stderr
