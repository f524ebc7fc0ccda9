"""bench.py's whole-pass refinement of launch shapes (refine_in_pass), run on
the host with a stand-in path whose pass time is a table of its shapes: the
descent keeps a shape only when whole passes get at least 0.5% faster, and
leaves every other step's shape as it found it."""
import types

import bench


class FakePath:
    """Two product steps; only some shapes are valid, as in the library."""

    def __init__(self):
        self.shapes = {10: (3, 1, 0), 11: (4, 1, 0)}
        self.valid = {10: {(3, 1, 0), (6, 1, 0), (6, 2, 0), (3, 1, 1)}, 11: {(4, 1, 0), (7, 1, 0)}}

    def gemm_configs(self, precision="c64"):
        return dict(self.shapes)

    def set_gemm_config(self, s, tile, split, tr=0, precision="c64"):
        if (tile, split, tr) not in self.valid[s]:
            raise bench_tnq.TNError("invalid shape")
        self.shapes[s] = (tile, split, tr)


class _Err(Exception):
    pass


bench_tnq = types.SimpleNamespace(TNError=_Err)


def run_refine(cost, monkeypatch):
    clock = [0.0]
    monkeypatch.setattr(bench.time, "perf_counter", lambda: clock[0])
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    path = FakePath()

    def run(p):
        clock[0] += cost(p.shapes) * 1e-3

    before, after, changed = bench.refine_in_pass(bench_tnq, fake_torch, path, run, "c64")
    return path, before, after, changed


def test_keeps_only_real_gains(monkeypatch):
    def cost(sh):  # ms per pass
        t = 1.0
        t -= {(6, 1, 0): 0.10, (6, 2, 0): 0.002, (3, 1, 1): 0.0}.get(sh[10], 0.0)
        t -= 0.003 if sh[11] == (7, 1, 0) else 0.0  # 0.3%: below the 0.5% bar
        return t

    path, before, after, changed = run_refine(cost, monkeypatch)
    assert path.shapes == {10: (6, 1, 0), 11: (4, 1, 0)}
    assert changed == 1
    assert abs(before - 1.0) < 1e-9 and abs(after - 0.9) < 1e-9


def test_no_change_restores_shapes(monkeypatch):
    path, before, after, changed = run_refine(lambda sh: 1.0 + 0.01 * (sh[10] != (3, 1, 0)), monkeypatch)
    assert path.shapes == {10: (3, 1, 0), 11: (4, 1, 0)}
    assert changed == 0 and before == after


def test_noise_only_gain_is_rejected(monkeypatch):
    """A candidate that looks faster once (a lucky timing) but is not faster
    when timed again against the current shape is not kept."""
    seen = {"n": 0}

    def cost(sh):
        if sh[10] == (6, 1, 0):
            seen["n"] += 1
            # the search's first timings of this shape are lucky, later ones are not
            return 0.9 if seen["n"] <= 4 else 1.0
        return 1.0

    path, before, after, changed = run_refine(cost, monkeypatch)
    assert path.shapes == {10: (3, 1, 0), 11: (4, 1, 0)}
    assert changed == 0 and abs(after - 1.0) < 1e-9
