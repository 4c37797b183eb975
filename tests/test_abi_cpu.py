"""CPU-only checks of the C ABI library and of the driver's host logic."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import mpo_oracle as mo
from paper_2604_21908_amd import circuitgen as cg
from paper_2604_21908_amd import driver as dr
from paper_2604_21908_amd import mpo as mpolib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "mpo.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpo_[a-z_]+)\s*\(", text)))


def ensure_built():
    if not os.path.exists(mpolib.LIB_PATH):
        from paper_2604_21908_amd import build
        build.build()


def test_library_exports_every_declared_symbol():
    ensure_built()
    lib = ctypes.CDLL(mpolib.LIB_PATH)
    names = header_functions()
    assert "mpo_init_identity" in names and "mpo_extract_peak" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(mpolib.EXPORTED) == names


def test_binding_loads_and_reports_version():
    ensure_built()
    lib = mpolib.load_library()
    assert b"gfx950" in lib.mpo_version()


def test_invalid_config_rejected_without_device():
    ensure_built()
    lib = mpolib.load_library()
    h = ctypes.c_void_p()
    bad = mpolib.MpoConfig(1, 8, 1e-12, 0, 0, 0, 0.0)            # n < 2
    assert lib.mpo_init_identity(ctypes.byref(bad), None, ctypes.byref(h)) == -1
    bad = mpolib.MpoConfig(4, 0, 1e-12, 0, 0, 0, 0.0)            # chi_max < 1
    assert lib.mpo_init_identity(ctypes.byref(bad), None, ctypes.byref(h)) == -1
    bad = mpolib.MpoConfig(4, 8, 1e-12, 7, 0, 0, 0.0)            # bad cutoff mode
    assert lib.mpo_init_identity(ctypes.byref(bad), None, ctypes.byref(h)) == -1
    assert lib.mpo_unswap_sweep(None, None, None, 0, None) == -1
    assert lib.mpo_extract_peak(None, None, None, None) == -1
    assert lib.mpo_tau_reached(None, None, None) == -1
    assert lib.mpo_trial_swap(None, 0, 0, None) == -1
    assert lib.mpo_counters(None, None, 0) == -1


def test_admission_by_projected_memory():
    """Serving admission (first come first served, n chi^2 16 B per request):
    the head is admitted while it fits, later requests never overtake it, and
    a request larger than the whole budget is refused."""
    from paper_2604_21908_amd import serve as sv
    R = sv.Request
    q = [R(0.0, 24, 6, 1), R(0.1, 56, 14, 2), R(0.2, 24, 6, 3), R(0.3, 200, 50, 4)]
    budget = sv.projected_bytes(24, 512) + sv.projected_bytes(40, 512)
    adm, ref, wait = sv.admit(q, 0, budget, 8, 512)
    assert [r.seed for r in adm] == [1] and [r.seed for r in ref] == [4] and [r.seed for r in wait] == [2, 3]
    adm, ref, wait = sv.admit(wait, 0, budget, 8, 512)
    assert [r.seed for r in adm] == [2] and [r.seed for r in wait] == [3]
    adm, ref, wait = sv.admit([R(0, 24, 6, 5), R(0, 24, 6, 6)], 0, budget, 1, 512)
    assert [r.seed for r in adm] == [5] and [r.seed for r in wait] == [6]


# ------------------------------------------------------------ host logic
def test_time_layers_and_split_match_the_oracle():
    c = cg.mirrored_peaked_circuit(9, 4, 5)
    a = dr.time_layers(c.gates, c.n)
    b = mo.asap_layers(c.gates, c.n)
    assert [[(g[0], g[1]) for g in l] for l in a] == [[(g[0], g[1]) for g in l] for l in b]


@pytest.mark.parametrize("router", ["up", "middle"])
def test_plan_step_matches_the_oracle_update_sequence(router):
    """The driver's ordered update list (routing, fusion, orientation) equals
    the oracle's on layouts scrambled by random swaps, under both routing
    rules."""
    rng = np.random.default_rng(0)
    for trial in range(20):
        n = int(rng.integers(4, 10))
        c = cg.mirrored_peaked_circuit(n, 3, 100 + trial)
        layers = dr.time_layers(c.gates, n)
        lg, rg = layers[len(layers) // 2], layers[len(layers) // 2 - 1]
        out_w, in_w = dr.Wires(n), dr.Wires(n)
        ct = mo.Contraction(n, [], mo.OracleConfig(router=router))
        for _ in range(int(rng.integers(0, 3 * n))):
            j = int(rng.integers(0, n - 1))
            if rng.random() < 0.5:
                out_w.exchange(j)
                ct.lay_l.swap_sites(j)
            else:
                in_w.exchange(j)
                ct.lay_r.swap_sites(j)
        ups = dr.plan_step(lg, rg, out_w, in_w, router)
        seen = []
        ct._update = lambda i, go, gi, stage, fused=False: seen.append((i, go, gi, stage))
        ct.left, ct.right = [lg], [rg]
        ct.absorb_step()
        assert len(seen) == len(ups)
        for u, (i, go, gi, stage) in zip(ups, seen):
            assert u.bond == i and u.stage == stage
            for x, y in ((u.g_out, go), (u.g_in, gi)):
                assert (x is None) == (y is None)
                if x is not None:
                    assert np.allclose(x, y)
        assert list(out_w.site_of) == ct.lay_l.site_of and list(in_w.site_of) == ct.lay_r.site_of


def test_wave_split_respects_dependencies():
    rng = np.random.default_rng(1)
    for _ in range(200):
        bonds = list(rng.integers(0, 12, size=int(rng.integers(1, 40))))
        waves = dr.wave_split(bonds)
        where = {}
        for w, idxs in enumerate(waves):
            bs = sorted(bonds[i] for i in idxs)
            assert all(b2 - b1 >= 2 for b1, b2 in zip(bs, bs[1:]))
            for i in idxs:
                where[i] = w
        assert sorted(where) == list(range(len(bonds)))
        for i in range(len(bonds)):
            for j in range(i):
                if abs(bonds[i] - bonds[j]) <= 1:
                    assert where[j] < where[i]


def test_binding_loads_a_single_hip_runtime():
    """Loading libmpo before anything else imports torch must still leave one
    HIP runtime in the process (torch's), so torch streams are valid in libmpo."""
    import subprocess
    import sys
    code = ("from paper_2604_21908_amd import mpo\n"
            "mpo.load_library()\n"
            "import torch\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
