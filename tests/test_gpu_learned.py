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
    hist, _ = learned.train(net, X, Y, epochs=6, batch=16, lr=1e-3)
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
        # same start and step size as the plain run, which is charged up to
        # its first step at the final error (the dose can differ in its last
        # bits: the deposit's FP64 sums are not ordered)
        assert r_["learned_steps"] <= r_["plain_steps"] + 1
        assert r_["plain_steps"] <= len(r_["plain_dose_errors"])
        assert min(r_["plain_dose_errors"][:r_["plain_steps"]]) <= r_["target_dose_error"]
    net.close()


def test_checkpoint_resume_matches_uninterrupted_training(tmp_path):
    # training split at a checkpoint (parameters, Adam moments and step
    # count, schedule position) takes exactly the steps of training that
    # never stopped
    import numpy as np
    rng = synth.SplitMix64(61)
    X = torch.from_numpy(rng.uniform(64 * 2 * 32 * 32).reshape(64, 2, 32, 32).astype(np.float32)).to("cuda:0")
    Y = X[:, 1] + 0.1 * X[:, 0]
    Y = Y.contiguous()
    a = Cnn(3, 16, 32, 32, max_batch=8, in_scale=(1.0, 1.0))
    a.set_params(synth.cnninit.he_init(3, 16, seed=4))
    _, step = learned.train(a, X, Y, epochs=2, batch=8, lr=1e-3, seed=0, total_steps=24)
    _, _ = learned.train(a, X, Y, epochs=1, batch=8, lr=1e-3, seed=1, step0=step, total_steps=24)
    b = Cnn(3, 16, 32, 32, max_batch=8, in_scale=(1.0, 1.0))
    b.set_params(synth.cnninit.he_init(3, 16, seed=4))
    _, step_b = learned.train(b, X, Y, epochs=2, batch=8, lr=1e-3, seed=0, total_steps=24)
    path = str(tmp_path / "ck.npz")
    learned.save_checkpoint(path, b, step_b, 24, 1.0, 1.0, {"test": 1})
    b.close()
    ck = learned.load_checkpoint(path)
    assert ck["step"] == step_b == 16 and ck["adam_steps"] == 16 and ck["meta"] == {"test": 1}
    c = Cnn(3, 16, 32, 32, max_batch=8, in_scale=(ck["s0"], ck["s1"]))
    c.set_state(ck["state"], ck["adam_steps"])
    state, t = c.get_state()
    assert t == 16 and np.array_equal(state, ck["state"])
    learned.train(c, X, Y, epochs=1, batch=8, lr=1e-3, seed=1, step0=ck["step"], total_steps=24)
    assert np.array_equal(a.get_params(), c.get_params())
    a.close()
    c.close()
