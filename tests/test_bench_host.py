"""Host checks of bench.py's timing structure (no GPU): the warm-up steps run
before the clock and the profiler start, exactly K steps are timed and
counted, and a request for more than one GPU is refused."""

import hashlib
import subprocess
import sys
import time
import types

import pytest
import torch

import bench


class FakeLib:
    """Stands in for the binding: records the order of steps and profiler calls."""

    def __init__(self):
        self.events = []
        self.profiling = False

    def llg_step_midpoint(self, ctx, prm, m, vh, lam, **kw):
        self.events.append(("step", self.profiling))
        time.sleep(0.002)
        return dict(picard_iters=5, lin_iters_total=48, max_len_err=0.0, converged=1)

    def llg_profile_select(self, ctx, kinds):
        pass

    def llg_profile_enable(self, ctx, on):
        self.profiling = bool(on)
        self.events.append(("profile", self.profiling))

    def llg_profile_read(self, ctx):
        return {"xinv_dots": dict(launches=1, total_ms=1.0, bytes=1e6)}


@pytest.fixture
def no_device(monkeypatch):
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)


def _runner(P, warmup, steps):
    spec = dict(scheme="midpoint", picard_tol=1e-10, picard_max=50, restart=30, rtol=1e-10, wid=4)
    ctx = types.SimpleNamespace(device="cpu")
    m0 = torch.zeros((3, 1, 2, 2), dtype=torch.float64)
    return bench.StepsRunner(P, ctx, None, m0, spec, "fp32_ir", warmup, steps, 1e-3, "dcgs2")


def test_warmup_steps_are_not_timed(no_device):
    P = FakeLib()
    r = _runner(P, warmup=5, steps=3)
    t, out = bench.timed_steps(r)
    assert len(out) == 3 and len(P.events) == 8
    # 3 steps of about 2 ms are timed, not the 8 that ran
    assert t < 7 * 0.002


def test_profiled_passes_time_and_profile_only_the_k_steps(no_device):
    P = FakeLib()
    r = _runner(P, warmup=2, steps=3)
    t, out, prof_all, prof = bench.profiled_timing(P, None, r, "test")
    assert len(out) == 3
    # three passes of (2 warm-up + 3 steps); the profiler is on during the 3
    # steps of the second and third passes only
    steps = [on for kind, on in P.events if kind == "step"]
    assert len(steps) == 15
    assert steps == [False] * 5 + [False] * 2 + [True] * 3 + [False] * 2 + [True] * 3
    assert bench.summarize(out, t, 3)["solves"] == 15


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert p.returncode != 0 and "one GPU" in (p.stdout + p.stderr)


def test_counter_traffic_is_reported_only_on_its_own_grid(monkeypatch, tmp_path):
    """A committed counter ratio belongs to the grid and the kernel source it
    was measured with: the roofline carries a traffic figure there and None on
    any other grid or once the source has changed."""
    src = tmp_path / "paper_2607_15290_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "k.h").write_text("kernel source")
    h = hashlib.sha256(b"kernel source").hexdigest()[:16]
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_3d256_midpoint.md").write_text(
        f"bench-traffic: xfwd_upd 1.0028 k.h {h} 256x256x256\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_COPY_GBS", 5000.0)  # the context copy needs a GPU
    assert bench.measured_traffic("xfwd_upd", 1e9, (256, 256, 256)) == pytest.approx(1.0028e9)
    for grid in ((128, 128, 128), (256, 256, 1), (512, 512, 512)):
        assert bench.measured_traffic("xfwd_upd", 1e9, grid) is None, grid
    assert bench.measured_traffic("no_such_kind", 1e9, (256, 256, 256)) is None
    prof = {"xfwd_upd": dict(launches=2, total_ms=1.0, bytes=2e9),
            "axis_fwd": dict(launches=4, total_ms=0.5, bytes=1e9)}
    big = 256 ** 3 * 128
    r = bench.roofline_of(prof, big, (256, 256, 256))
    assert r["kernel"] == "xfwd_upd" and r["traffic"] == round(1.0028e9)
    assert bench.roofline_of(prof, big, (128, 128, 128))["traffic"] is None
    (src / "k.h").write_text("kernel source, edited")
    assert bench.measured_traffic("xfwd_upd", 1e9, (256, 256, 256)) is None
