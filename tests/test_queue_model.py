"""Host model of the persistent batch kernel's work queue (CPU only).

tests/model/queue_model.cpp runs the kernel's own claim / wait / publish code
(paper_1508_05610_amd/csrc/lf2_queue.hpp, item order from lf2_batch_items.hpp)
on std::threads, with fewer resident blocks than blocks, under
ThreadSanitizer.  The shipped protocol must finish every item once with no
wait giving up, no race and the queue reset; the two ways such a kernel can
hang -- a fixed block-to-item assignment while not every block is resident,
and items handed out in an order that is not a dependency order -- must
show up as waits that give up (the bounded spin), not as a hang; a queue no
block serves shows up in the error word.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "model", "queue_model.cpp")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    d = tmp_path_factory.mktemp("qmodel")
    tsan = str(d / "qm_tsan")
    plain = str(d / "qm")
    base = ["g++", "-std=c++20", "-O1", "-g", "-pthread", SRC]
    subprocess.check_call(base + ["-fsanitize=thread", "-o", tsan])
    subprocess.check_call(base + ["-o", plain])
    return tsan, plain


def run(binary, *args, timeout=240):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([binary, *map(str, args)], capture_output=True, text=True,
                       timeout=timeout, env=env)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.parametrize("blocks,resident,threads,seed,fields,queues", [
    (64, 64, 4, 1, 8, 8),     # every block resident, one queue per XCD
    (64, 3, 4, 2, 8, 8),      # few resident blocks: items wait on blocks that started earlier
    (32, 1, 4, 3, 6, 4),      # one block at a time
    (200, 17, 2, 4, 48, 8),   # the 48-field batch shape, residency well below the grid
    (96, 96, 8, 5, 48, 1),    # one queue for all blocks
])
def test_ticket_protocol_completes_race_free(binaries, blocks, resident, threads, seed, fields,
                                             queues):
    rc, out = run(binaries[0], "ticket", blocks, resident, threads, seed, fields, queues)
    print(out.strip().splitlines()[-1])
    assert "ThreadSanitizer" not in out, out
    assert rc == 0, out
    assert "errors=0" in out and "reset=1" in out


def test_static_assignment_deadlocks_below_full_residency(binaries):
    """Block b taking items b, b + G, ... waits on items of blocks that cannot
    start until it ends: only the bounded spin ends the wait."""
    rc, out = run(binaries[1], "static", 16, 2, 4, 5, 4)
    print(out.strip().splitlines()[-1])
    assert rc == 1 and "errors=1" in out


def test_non_dependency_order_deadlocks(binaries):
    rc, out = run(binaries[1], "reverse", 16, 16, 4, 6, 4, 2)
    print(out.strip().splitlines()[-1])
    assert rc == 1 and "errors=1" in out


def test_queue_without_blocks_is_reported(binaries):
    """A queue that no block serves leaves items unclaimed: error bit 1, no wait."""
    rc, out = run(binaries[1], "starved", 16, 16, 4, 7, 8, 4)
    print(out.strip().splitlines()[-1])
    assert rc == 1 and "errors=2" in out


def test_runtime_radix_schedules(tmp_path):
    """Host check of the run-time radix schedules (tests/model/sched_check.cpp)."""
    exe = str(tmp_path / "sched_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-o", exe,
                           os.path.join(ROOT, "tests", "model", "sched_check.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout.strip())
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout
