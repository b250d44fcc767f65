"""The trainer's checkpoint file round trip on the host: the training state
handed to the model, the batch-order generator, counters, history and the
best parameters so far come back exactly (the model is a stand-in that only
keeps what it is given)."""
import numpy as np

from paper_2509_01416_amd import train as T


class _Model:
    def __init__(self, state):
        self.state = state

    def get_state(self):
        return self.state

    def set_state(self, state):
        self.state = state


def test_checkpoint_round_trip(tmp_path):
    rng = np.random.Generator(np.random.PCG64(5))
    rng.permutation(100)                      # advance the generator
    n = 17
    st = dict(params=np.arange(n, dtype=np.float32), adam_m=np.full(n, 0.5, np.float32),
              adam_v=np.full(n, 0.25, np.float32), step=1234)
    best = (3.5e-3, 40, np.linspace(0, 1, n).astype(np.float32))
    hist = [dict(epoch=5, train_mse=1.0, val_rel_l2_mean=0.1, seconds=2.0)]
    path = str(tmp_path / "ck.npz")
    T.save_checkpoint(path, _Model(st), rng, 45, 2535, best, hist)
    want_next = rng.permutation(100)
    m = _Model(None)
    rng2 = np.random.Generator(np.random.PCG64(99))
    epoch, steps, best2, hist2 = T.load_checkpoint(path, m, rng2)
    assert (epoch, steps) == (45, 2535) and hist2 == hist
    assert best2[0] == best[0] and best2[1] == best[1] and np.array_equal(best2[2], best[2])
    for k in ("params", "adam_m", "adam_v"):
        assert np.array_equal(m.state[k], st[k])
    assert m.state["step"] == 1234
    assert np.array_equal(rng2.permutation(100), want_next)
