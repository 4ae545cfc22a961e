"""Every global access of the estimator kernels stays inside its allocation.

Host only: ``tests/replay/address_replay.cpp`` builds the launches of
estimator calls and of served request slots with the library's own host
plan (``csrc/plan.cpp``) over a synthetic address space and replays each
kernel's load and store addresses (sweep, BF16 and FP64 low-rank kernels,
FP64 projection, init, reduction; single and batched launches).  Cases: the
benchmark workloads at full size (n = 256, 4,096, 16,384, 65,536 with rank
profiles zero, at the cap, full and random), the serving stream's request
sizes, the no-allocation region, requested chunk sizes, slices of the
sample range, two worker streams, and a grid of small problems (ragged
tiles, every form, odd sample counts) replayed thread by thread.  Planted
mistakes (a short buffer, a map entry past Z) must be reported.
"""

from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2003_11183_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "replay", "address_replay.cpp")

# case-name prefixes run by one process each
GROUPS = [
    "cfg1", "cfg2", "cfg3", "cfg4", "serve-n1 serve-n4", "serve-n9", "streams noalloc",
    "small-c small-s small-no small-n1- small-n2- small-n15- small-n17-", "small-n100-", "small-n333-",
    "small-n1000-",
]


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("clang++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("replay") / "address_replay")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC, SRC,
                    os.path.join(CSRC, "plan.cpp"), "-o", exe], check=True)
    return exe


def _run(exe, prefixes):
    p = subprocess.run([exe, *prefixes.split()], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600)
    return prefixes, p.returncode, p.stdout


def test_every_kernel_access_stays_inside_its_allocation(replay):
    workers = max(1, min(len(GROUPS), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda g: _run(replay, g), GROUPS))
    cases = 0
    for prefixes, rc, out in results:
        assert rc == 0, f"replay of {prefixes!r} failed:\n{out[-4000:]}"
        last = out.strip().splitlines()[-1]
        assert "outside their allocation 0" in last, out[-2000:]
        cases += int(last.split()[1])
    assert cases > 800  # every case of every group ran


def test_planted_mistakes_are_reported(replay):
    _, rc, out = _run(replay, "plant-")
    assert rc == 0, out
    lines = [ln for ln in out.splitlines() if ln.startswith("plant-")]
    assert len(lines) == 4 and all(ln.endswith("caught") for ln in lines), out
    assert "planted mistakes 4, caught 4" in out
