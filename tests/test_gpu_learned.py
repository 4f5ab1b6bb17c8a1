"""The learned initialiser end to end at a reduced size (64^3 grid, 64^2
DMD, 60 angles, c5 optics scaled by 1/2): data from the plain ray-traced
optimisation of 24 seeded targets, MFMA training, and evaluation on 4
held-out targets by the ray-traced projector.  The trained network must
start closer to the target dose than the plain filtered start and reach the
plain method's final dose error in fewer optimisation steps."""
import sys

import pytest

import synth

torch = pytest.importorskip("torch")
from paper_2211_03516_amd import learned, Cnn

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_learned_start_beats_plain_start():
    p = synth.workload("c5")
    r = 0.5
    p = synth.configs.scaled(p, nx=64, ny=64, nz=64, nu=64, nv=64, n_angles=60, r_outer=p["r_outer"] * r,
                             r_inner=p["r_inner"] * r, focus=p["focus"] * r, pupil=p["pupil"] * r)
    fn = synth.random_config2_target
    X, Y = learned.make_dataset(p, list(range(1000, 1024)), 15, fn)
    s0 = 1.0 / float(X[:, 0].abs().max())
    s1 = 1.0 / float(X[:, 1].abs().mean())
    net = Cnn(6, 32, 64, 64, max_batch=16, in_scale=(s0, s1))
    net.set_params(synth.cnninit.he_init(6, 32, seed=0))
    hist = learned.train(net, X, Y, epochs=6, batch=16, lr=1e-3)
    say("training loss per epoch", ["%.4f" % h for h in hist])
    assert hist[-1] < hist[0]
    rows = learned.evaluate(net, p, list(range(5000, 5004)), 15, fn, 16, log=say)
    s = learned.summarise(rows)
    say(s)
    assert s["mean_dose_error_learned_start"] < s["mean_dose_error_plain_start"]
    assert s["reached"] == len(rows)
    assert s["mean_learned_steps"] < s["mean_plain_steps"]
    net.close()


def test_fallback_to_the_plain_start():
    # a network whose output is far from any useful start must not be used:
    # the evaluation falls back to the filtered start and then follows the
    # plain method
    p = synth.workload("c5")
    r = 0.5
    p = synth.configs.scaled(p, nx=64, ny=64, nz=64, nu=64, nv=64, n_angles=60, r_outer=p["r_outer"] * r,
                             r_inner=p["r_inner"] * r, focus=p["focus"] * r, pupil=p["pupil"] * r)
    net = Cnn(3, 8, 64, 64, max_batch=16, in_scale=(1.0, 1.0))
    bad = synth.cnninit.he_init(3, 8, seed=1, zero_last=False)
    last = synth.cnninit.param_count(3, 8) - (1 * 9 * 8 + 1)
    bad[last:] = -50.0                     # last layer: a large negative offset (dose < 0 everywhere)
    net.set_params(bad)
    rows = learned.evaluate(net, p, [5100, 5101], 8, synth.random_config2_target, 16, log=say)
    for r_ in rows:
        assert r_["fallback"]
        assert r_["dose_error_learned_start"] > r_["dose_error_plain_start"]
        # same start and step size as the plain run (the dose can differ in
        # its last bits: the deposit's FP64 sums are not ordered)
        assert r_["learned_steps"] <= r_["plain_steps"]
    net.close()
