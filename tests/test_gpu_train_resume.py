"""Training checkpoints: a run interrupted after 3 steps and resumed from
its checkpoint (fp32 masters, Adam moments and step, the pool of human
configurations, both random generators, the schedule) ends with the same
parameters, bit for bit, as the uninterrupted 6-step run; and training on
the GPU's own labels lowers the loss."""
import sys

import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_grid():
    return scenegen.Grid(72, 64, 48, 0.04)


def test_resume_continues_exactly(dev, tmp_path):
    from paper_2201_05058_amd.train import Trainer
    g = small_grid()
    kw = dict(pool=4, batch=2048, steps=6, seed=3)
    say("train resume: 6 straight steps")
    a = Trainer(g, dev, **kw)
    a.init_network()
    a.run(log=lambda s: None)
    pa = a.net.get_params()
    say("train resume: 3 steps, checkpoint, resume, 3 steps")
    b = Trainer(g, dev, **kw)
    b.init_network()
    b.run(until=3, log=lambda s: None)
    ck = str(tmp_path / "ck.npz")
    b.save_checkpoint(ck)
    b.net.close()
    c = Trainer.resume(ck, g, dev)
    assert c.step == 3
    c.run(log=lambda s: None)
    np.testing.assert_array_equal(c.net.get_params(), pa)
    np.testing.assert_array_equal(c.xy, a.xy)
    assert c.net.get_state()[3] == 6
    a.net.close()
    c.net.close()


def test_training_lowers_the_loss(dev):
    """The loss ends well below the targets' variance (the loss of the best
    constant prediction)."""
    from paper_2201_05058_amd.train import Trainer
    t = Trainer(small_grid(), dev, pool=8, batch=8192, steps=1500, seed=5)
    t.init_network()
    _, tg = t.batch_rows(65536)
    var = float(tg.double().var())
    t.run(log=lambda s: None, log_every=100)
    hist = [l for _, l in t.hist]
    say("target variance", var, "loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.4 * var
    t.net.close()
