"""The plan cache of the stepper autotuner (host logic, no GPU): first use tunes and stores, later uses apply the
stored plan, and the key separates problems that may want different plans."""
from paper_2008_10904_amd import autotune


class FakeOp:
    def __init__(self, n, offsets, precision):
        self.n, self.offsets, self.precision = n, offsets, precision
        self.tuned, self.applied = 0, []

    def tune(self, k, steps):
        self.tuned += 1
        return (12, 128, 16, 1), 0.33

    def set_plan(self, plan):
        self.applied.append(tuple(plan))
        return tuple(plan)


def test_cache_tunes_once_then_applies(tmp_path):
    path = str(tmp_path / "plans.json")
    op = FakeOp(2000, [0, 2000], "fp64")
    plan, us = autotune.tuned(op, 4, device="dev", path=path)
    assert plan == (12, 128, 16, 1) and us == 0.33 and op.tuned == 1
    plan, us = autotune.tuned(op, 4, device="dev", path=path)
    assert us is None and op.tuned == 1 and op.applied == [(12, 128, 16, 1)]
    autotune.tuned(op, 4, device="dev", path=path, retune=True)
    assert op.tuned == 2


def test_cache_key_separates_problems(tmp_path):
    path = str(tmp_path / "plans.json")
    a = FakeOp(2000, [0, 2000], "fp64")
    autotune.tuned(a, 4, device="dev", path=path)
    for other, k in ((FakeOp(2000, [0, 2000], "mixed"), 4), (FakeOp(2000, [0, 2000], "fp64"), 2),
                     (FakeOp(2000, [0, 1000, 2000], "fp64"), 4)):
        autotune.tuned(other, k, device="dev", path=path)
        assert other.tuned == 1
    assert len(autotune.load(path)) == 4


def test_cache_survives_a_corrupt_file(tmp_path):
    path = tmp_path / "plans.json"
    path.write_text("{not json")
    op = FakeOp(300, [0, 300], "fp64")
    autotune.tuned(op, 1, device="dev", path=str(path))
    assert op.tuned == 1 and len(autotune.load(str(path))) == 1


class FakePowerOp(FakeOp):
    """Step power 4 is fastest for this fake operator."""

    def __init__(self, *a):
        super().__init__(*a)
        self.power = 4

    def set_step_power(self, m):
        self.power = m

    def get_step_power(self):
        return self.power

    def tune(self, k, steps):
        self.tuned += 1
        return (10, 256, 32, 1) if self.power == 4 else (12, 128, 16, 1), {4: 0.24, 2: 0.29, 1: 0.35}[self.power]


def test_cache_chooses_the_step_power(tmp_path):
    path = str(tmp_path / "plans.json")
    op = FakePowerOp(2000, [0, 2000], "fp64")
    op.power = 1
    plan, us = autotune.tuned(op, 4, device="dev", path=path, powers=(1, 2, 4))
    assert op.tuned == 3 and op.power == 4 and plan == (10, 256, 32, 1) and us == 0.24
    op.power = 1
    plan, us = autotune.tuned(op, 4, device="dev", path=path, powers=(1, 2, 4))
    assert us is None and op.tuned == 3 and op.power == 4 and plan == (10, 256, 32, 1)
    # a fixed-power entry is kept apart from the power search
    op.power = 2
    autotune.tuned(op, 4, device="dev", path=path)
    assert op.tuned == 4 and op.power == 2 and len(autotune.load(path)) == 2
