"""Host side of the fault-tolerant chain driver (Sec. III: every process
periodically records its step count, running mean and uncertainty, so a job
killed at any time loses nothing and can be restarted): atomic checkpoint
files, the choice of the checkpoint to resume from when the newest one is
torn or damaged, the block records, and a writer killed with SIGKILL in the
middle of its checkpoint stream.  No GPU: the checkpoint payloads here are
synthetic arrays of the right layout."""
import json
import os
import signal
import subprocess
import sys
import time

import numpy as np

from paper_2203_05632_amd.chain import (CHECKPOINT_FORMAT, atomic_savez, checkpoint_path, latest_checkpoint,
                                        read_checkpoint, read_records, truncate_records)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _state(step, want_grad=False, n=4):
    st = {"format": np.int64(CHECKPOINT_FORMAT), "walkers": np.full((n, 2, 3), step, dtype=float),
          "w": np.ones(n), "key": np.array([3, 1]), "step": np.int64(step), "n_burn": np.int64(10),
          "delta": np.float64(0.4), "n_tau": np.int64(2), "values": np.arange(3.0 * step).reshape(step, 3),
          "want_grad": np.bool_(want_grad), "accepted": np.int64(step), "proposed": np.int64(4 * step)}
    if want_grad:
        for k in ("eps_s", "eps_c", "c_s", "c_c"):
            st["acc_" + k] = np.zeros(5)
    return st


def test_atomic_save_roundtrip_and_no_temporary_left(tmp_path):
    p = checkpoint_path(str(tmp_path), 100)
    atomic_savez(p, **_state(100, want_grad=True))
    st = read_checkpoint(p)
    assert st is not None and int(st["step"]) == 100 and bool(st["want_grad"])
    assert sorted(os.listdir(tmp_path)) == [os.path.basename(p)]


def test_incomplete_files_are_not_checkpoints(tmp_path):
    d = str(tmp_path)
    atomic_savez(checkpoint_path(d, 100), **_state(100))
    atomic_savez(checkpoint_path(d, 200), **_state(200))
    # a newer file torn in the middle of writing, and a temporary file of an interrupted save
    good = open(checkpoint_path(d, 200), "rb").read()
    with open(checkpoint_path(d, 300), "wb") as fh:
        fh.write(good[: len(good) // 2])
    with open(os.path.join(d, ".chain-000000000400.npz.999.tmp"), "wb") as fh:
        fh.write(good[:100])
    assert read_checkpoint(checkpoint_path(d, 300)) is None
    assert latest_checkpoint(d) == checkpoint_path(d, 200)
    # a gradient checkpoint without its accumulators, or another format, is rejected
    st = _state(500, want_grad=True)
    del st["acc_c_s"]
    np.savez(checkpoint_path(d, 500), **st)
    st = _state(600)
    st["format"] = np.int64(CHECKPOINT_FORMAT - 1)
    np.savez(checkpoint_path(d, 600), **st)
    assert latest_checkpoint(d) == checkpoint_path(d, 200)
    assert latest_checkpoint(str(tmp_path / "empty")) is None


def test_records_truncate_to_the_checkpoint(tmp_path):
    d = str(tmp_path)
    with open(os.path.join(d, "records.jsonl"), "w") as fh:
        for n in (100, 200, 300):
            fh.write(json.dumps({"N": n, "I_N": [0.0, 0.0, float(n)]}) + "\n")
        fh.write('{"N": 400, "I_N": [0.0')          # torn last line
    assert [r["N"] for r in read_records(d)] == [100, 200, 300]
    truncate_records(d, 200)
    assert [r["N"] for r in read_records(d)] == [100, 200]


WRITER = r"""
import sys, time
sys.path.insert(0, {root!r})
import numpy as np
from paper_2203_05632_amd.chain import CHECKPOINT_FORMAT, atomic_savez, checkpoint_path
d = {d!r}
step = 0
while True:
    step += 1
    st = {{"format": np.int64(CHECKPOINT_FORMAT), "walkers": np.full((64, 2, 3), step, dtype=float),
          "w": np.ones(64), "key": np.array([3, 1]), "step": np.int64(step), "n_burn": np.int64(0),
          "delta": np.float64(0.5), "n_tau": np.int64(1),
          "values": np.full((step, 3), float(step)), "want_grad": np.bool_(False),
          "accepted": np.int64(0), "proposed": np.int64(0)}}
    atomic_savez(checkpoint_path(d, step), **st)
    print(step, flush=True)
"""


def test_writer_killed_mid_stream_leaves_a_complete_checkpoint(tmp_path):
    """SIGKILL a process that writes checkpoints back to back: the newest
    complete checkpoint is self-consistent (its payload matches its step)."""
    d = str(tmp_path)
    proc = subprocess.Popen([sys.executable, "-c", WRITER.format(root=ROOT, d=d)], stdout=subprocess.PIPE)
    deadline = time.time() + 60
    while time.time() < deadline:      # wait until a few checkpoints exist, then kill at once
        if len([f for f in os.listdir(d) if f.startswith("chain-")]) >= 20:
            break
        time.sleep(0.01)
    os.kill(proc.pid, signal.SIGKILL)
    proc.wait()
    path = latest_checkpoint(d)
    assert path is not None
    st = read_checkpoint(path)
    step = int(st["step"])
    assert path == checkpoint_path(d, step)
    assert st["values"].shape == (step, 3) and np.all(st["values"] == step)
    assert np.all(st["walkers"] == step)
