"""Host-side logic that needs no GPU: the PCG tuning table of the binding."""
import json

from paper_1808_05510_amd import connreg


class FakeProblem:
    """Stands in for connreg.Problem: records autotune and set_tuning calls."""

    def __init__(self, n_y, n_x, n_inj, precision="mixed", vpt=(1, 2)):
        self.n_y, self.n_x, self.n_inj, self.precision = n_y, n_x, n_inj, precision
        self.vpt = vpt
        self.tuned = 0
        self.set = None

    def autotune(self, cu_share=0):
        self.tuned += 1
        return self.vpt[0], self.vpt[1], 20.0, 30.0

    def set_tuning(self, vu, vv):
        self.set = (vu, vv)


def test_bucket_groups_sizes_by_half_octave_and_injection_block():
    a = FakeProblem(64000, 27000, 64)
    b = FakeProblem(66000, 26500, 61)  # same half-octaves, same 16-injection block
    c = FakeProblem(91000, 27000, 64)  # next half-octave of n_y
    d = FakeProblem(64000, 27000, 64, precision="fp64")
    T = connreg.TuningTable
    assert T.bucket(a) == T.bucket(b)
    assert T.bucket(a) != T.bucket(c)
    assert T.bucket(a) != T.bucket(d)
    assert T.bucket(a, 32) != T.bucket(a, 0)


def test_table_tunes_once_per_bucket_and_persists(tmp_path):
    path = str(tmp_path / "pcg_tuning.json")
    t = connreg.TuningTable(path)
    a = FakeProblem(64000, 27000, 64, vpt=(1, 2))
    e = t.apply(a)
    assert a.tuned == 1 and a.set == (1, 2) and e["vpt_v"] == 2
    b = FakeProblem(66000, 26500, 61, vpt=(8, 8))
    t.apply(b)
    assert b.tuned == 0 and b.set == (1, 2)  # reused, not re-timed
    with open(path) as f:
        saved = json.load(f)
    assert list(saved) == [connreg.TuningTable.bucket(a)]
    # a new table on the same file knows the bucket
    t2 = connreg.TuningTable(path)
    c = FakeProblem(64000, 27000, 64, vpt=(4, 4))
    t2.apply(c)
    assert c.tuned == 0 and c.set == (1, 2)
    # without tuning a new bucket is left alone
    d = FakeProblem(200000, 100000, 128)
    assert t2.apply(d, tune_missing=False) is None and d.set is None and d.tuned == 0
