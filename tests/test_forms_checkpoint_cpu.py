"""Host logic of the peak form's checkpoint: what _save_state writes,
_load_state restores on a fresh contraction of the same circuit (site
tensors, bond vectors, both wire layouts, the layers still to absorb, the
update count), with a stand-in for the device MPO.  CPU only."""
import types

import numpy as np

from paper_2604_21908_amd import driver as dr
from paper_2604_21908_amd import forms_bench as fb


class FakeMPO:
    def __init__(self, n, rng=None, dtype=np.complex128):
        self.n = n
        self.sites, self.lams = [], []
        if rng is not None:
            chis = [1] + [int(rng.integers(1, 5)) for _ in range(n - 1)] + [1]
            self.sites = [(rng.standard_normal((chis[i], 4, chis[i + 1]))
                           + 1j * rng.standard_normal((chis[i], 4, chis[i + 1]))).astype(dtype)
                          for i in range(n)]
            self.lams = [np.sort(rng.random(chis[b + 1]))[::-1] for b in range(n - 1)]

    def read_site(self, i):
        return self.sites[i].astype(np.complex128)

    def singular_values(self, b):
        return self.lams[b].copy()

    def load_state(self, sites, lams):
        self.sites = [np.asarray(s) for s in sites]
        self.lams = [np.asarray(l) for l in lams]


def fake_contractor(n, layers_left, layers_right, precision, mpo):
    c = types.SimpleNamespace()
    c.n = n
    c.cfg = dr.RunConfig(precision=precision)
    c.c_left = list(layers_left)
    c.c_right = list(layers_right)
    c.out_w, c.in_w = dr.Wires(n), dr.Wires(n)
    c.m = mpo
    c.bond_updates = 0
    return c


def test_checkpoint_round_trip(tmp_path):
    rng = np.random.default_rng(3)
    n = 6
    layers_l = [[("L", k)] for k in range(5)]
    layers_r = [[("R", k)] for k in range(3)]
    for prec, dt in (("fp64", np.complex128), ("mixed", np.complex64)):
        a = fake_contractor(n, layers_l, layers_r, prec, FakeMPO(n, rng, dt))
        for _ in range(2):                    # two absorption steps done
            a.c_left.pop(0)
            a.c_right.pop(0)
        a.out_w.exchange(1)
        a.out_w.exchange(3)
        a.in_w.exchange(2)
        a.bond_updates = 123
        path = str(tmp_path / f"ckpt_{prec}.npz")
        fb._save_state(path, a, 2, 4.5, 7)
        b = fake_contractor(n, layers_l, layers_r, prec, FakeMPO(n))
        steps, secs, max_k = fb._load_state(path, b)
        assert (steps, secs, max_k) == (2, 4.5, 7)
        assert b.c_left == layers_l[2:] and b.c_right == layers_r[2:]
        assert np.array_equal(b.out_w.site_of, a.out_w.site_of)
        assert np.array_equal(b.out_w.logical_at, a.out_w.logical_at)
        assert np.array_equal(b.in_w.site_of, a.in_w.site_of)
        assert b.bond_updates == 123
        for i in range(n):                    # exact, in the MPO's own precision
            assert b.m.sites[i].dtype == dt
            assert np.array_equal(b.m.sites[i], a.m.sites[i])
        for k in range(n - 1):
            assert np.array_equal(b.m.lams[k], a.m.lams[k])
