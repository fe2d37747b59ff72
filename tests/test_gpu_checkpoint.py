"""Checkpoint/resume, the caller's allocator, the Gauss-residual cadence and the step log, through the C ABI.

A run saved after some steps and restored into a fresh run on the same mesh
must take the following steps bit for bit as the saved run does, and saving
must not change the saved run.  The checks compare every state the ABI
exposes exactly (np.array_equal), not within a tolerance.
"""
import os

import numpy as np
import pytest

import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W

pytestmark = pytest.mark.gpu

QE, ME = -W.Q_E, W.M_E


def beam_setup(N=8, k=2, n=20000, seed=11):
    mesh = F.Mesh.cube(N, k)
    dt = 10 * mesh.info()["dt_cfl"]
    pos, vel = W.particles("beam", n, seed, vth=0.005, drift=0.1)
    return mesh, dt, pos, vel, W.plasma_weight(n, dt)


def state(run):
    e, b = run.fields()
    pos, vel, tet = run.particles()
    vh, ah = run.history()
    return dict(e=e, b=b, pos=pos, vel=vel, tet=tet, vh=vh, ah=ah, gauss=run.gauss())


def assert_same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("precision", [F.MIXED, F.FP64])
def test_resume_is_bitwise(tmp_path, precision):
    """8^3 cube, order 2, 20k-electron beam at 0.1c, dt = 10 dt_cfl: 6 steps, save, 6 more, against
    a fresh run restored from the file and stepped 6 times, and an uninterrupted 12-step run."""
    mesh, dt, pos, vel, w = beam_setup()
    path = str(tmp_path / "run.ckpt")
    a = F.Run(mesh, dt, precision, pcg_rtol=1e-14)
    a.load(pos, vel, QE, ME, w)
    a.step(6)
    a.save(path)
    a.step(6)
    sa = state(a)
    assert a.stats()["steps"] == 12 and a.stats()["crossings"] > 0
    b = F.Run(mesh, dt, precision, pcg_rtol=1e-14)
    b.restore(path)
    assert b.n == len(pos) and b.stats()["steps"] == 6
    b.step(6)
    assert b.stats()["steps"] == 12
    assert_same(sa, state(b))
    c = F.Run(mesh, dt, precision, pcg_rtol=1e-14)
    c.load(pos, vel, QE, ME, w)
    c.step(12)
    assert_same(sa, state(c))
    for r in (a, b, c):
        r.close()


def test_checkpoint_rejects_mismatch_and_damage(tmp_path):
    mesh, dt, pos, vel, w = beam_setup(n=5000)
    path = str(tmp_path / "run.ckpt")
    a = F.Run(mesh, dt, F.MIXED)
    a.load(pos, vel, QE, ME, w)
    a.step(2)
    a.save(path)
    blob = open(path, "rb").read()

    def rejected(run, p, what):
        with pytest.raises(F.FempicError) as ei:
            run.restore(p)
        assert ei.value.code == -1, what
        return str(ei.value)

    other_mesh = F.Run(F.Mesh.cube(6, 2), dt, F.MIXED)
    assert "mesh" in rejected(other_mesh, path, "mesh")
    assert "precision" in rejected(F.Run(mesh, dt, F.FP64), path, "precision")
    assert "time step" in rejected(F.Run(mesh, 0.5 * dt, F.MIXED), path, "dt")
    rejected(other_mesh, str(tmp_path / "missing.ckpt"), "missing file")
    short = str(tmp_path / "short.ckpt")
    open(short, "wb").write(blob[: len(blob) // 2])
    # the target keeps its own state after a failed restore
    b = F.Run(mesh, dt, F.MIXED)
    b.load(pos[:100], vel[:100], QE, ME, w)
    assert "truncated" in rejected(b, short, "truncated")
    flipped = bytearray(blob)
    flipped[len(blob) // 3] ^= 0x10
    bad = str(tmp_path / "bad.ckpt")
    open(bad, "wb").write(bytes(flipped))
    assert "checksum" in rejected(b, bad, "checksum")
    # a particle count far beyond the file (header field at byte 64) is caught before any allocation
    import struct
    big = bytearray(blob)
    big[64:72] = struct.pack("<q", (1 << 30) - 1)
    open(bad, "wb").write(bytes(big))
    msg = rejected(b, bad, "particle count")
    assert "wrong size" in msg or "header is corrupt" in msg, msg
    b.step(1)
    assert b.stats()["steps"] == 1 and b.stats()["n_particles"] == 100
    with pytest.raises(F.FempicError):
        F.Run(mesh, dt, F.MIXED).save(str(tmp_path / "empty.ckpt"))  # nothing loaded
    for r in (a, b, other_mesh):
        r.close()


TORCH_ALLOC_CHILD = r"""
import json, sys
import numpy as np
import torch  # first, so that the library binds to torch's HIP runtime
sys.path.insert(0, sys.argv[1])
import paper_2111_12411_amd as F
from paper_2111_12411_amd import workloads as W
mesh = F.Mesh.cube(8, 2)
dt = 10 * mesh.info()["dt_cfl"]
n = 20000
pos, vel = W.particles("beam", n, 11, vth=0.005, drift=0.1)
w = W.plasma_weight(n, dt)
def state(run):
    e, b = run.fields()
    p, v, t = run.particles()
    return [e, b, p, v, t, run.gauss()]
ref = F.Run(mesh, dt, F.MIXED, pcg_rtol=1e-14)
ref.load(pos, vel, -W.Q_E, W.M_E, w)
ref.step(4)
s_ref = state(ref)
ref.close()
torch.cuda.synchronize()
before = torch.cuda.memory_allocated()
F.use_torch_allocator()
run = F.Run(mesh, dt, F.MIXED, pcg_rtol=1e-14)
run.load(pos, vel, -W.Q_E, W.M_E, w)
during = torch.cuda.memory_allocated()
run.step(4)
same = all(np.array_equal(a, b) for a, b in zip(s_ref, state(run)))
run.close()
F.set_allocator()
torch.cuda.synchronize()
after = torch.cuda.memory_allocated()
print(json.dumps(dict(runtimes=F.hip_runtimes(), footprint=mesh.footprint(n, F.MIXED), before=before,
                      during=during, after=after, same=same)))
"""


def test_torch_allocator_holds_the_buffers_and_changes_nothing():
    """With torch's caching allocator installed, a run's device buffers come from torch (its
    allocated bytes grow by about the run's footprint and fall back after close) and the run's
    results are bit-identical to those of a run on hipMalloc memory.  torch has to be imported
    before the library is loaded, so this runs in a child process of its own."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", TORCH_ALLOC_CHILD, root], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert len(out["runtimes"]) == 1, out
    assert out["during"] - out["before"] > 0.5 * out["footprint"], out
    assert out["same"], out
    assert out["after"] <= out["before"] + (1 << 20), out


def test_gauss_cadence():
    """gauss_every = 3: the residuals of step 6 are in the statistics after 7 steps, equal to the
    ones fempic_gauss_residual returns at step 6."""
    mesh, dt, pos, vel, w = beam_setup(n=5000)
    run = F.Run(mesh, dt, F.FP64, pcg_rtol=1e-14, gauss_every=3)
    run.load(pos, vel, QE, ME, w)
    run.step(6)
    g6 = run.gauss()
    st = run.stats()
    assert st["gauss_step"] == 6 and np.array_equal(np.array(st["gauss"]), g6)
    run.step(1)
    st = run.stats()
    assert st["gauss_step"] == 6 and np.array_equal(np.array(st["gauss"]), g6)
    assert g6[0] < 1e-12
    run.close()


def test_step_log(tmp_path):
    """One JSON line per step: steps 1..5, the Gauss residuals on the steps gauss_every = 2 evaluates
    (equal to the statistics), the last step's counts equal to the statistics, and the per-step
    particle-phase times summing to the call's."""
    import json
    mesh, dt, pos, vel, w = beam_setup(n=5000)
    path = tmp_path / "steps.jsonl"
    run = F.Run(mesh, dt, F.MIXED, pcg_rtol=1e-14, gauss_every=2)
    run.load(pos, vel, QE, ME, w)
    run.set_log(str(path))
    run.step(5)
    st = run.stats()
    run.set_log(None)
    run.step(1)
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert [x["step"] for x in lines] == [1, 2, 3, 4, 5]
    assert ["gauss" in x for x in lines] == [False, True, False, True, False]
    assert lines[3]["gauss"] == st["gauss"] and st["gauss_step"] == 4
    last = lines[-1]
    for k in ("crossings", "reflections", "spills", "pcg_iters", "pcg_relres", "n_particles"):
        assert last[k] == st[k], k
    assert abs(sum(x["particle_ms"] for x in lines) - st["particle_ms"]) < 1e-3 * st["particle_ms"] + 1e-6
    assert all(x["field_ms"] > 0 and x["crossings"] > 0 for x in lines)
    run.close()
