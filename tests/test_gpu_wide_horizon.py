"""Horizons beyond LDS (the paper chooses delta up to 7h, Sec. 5): the local
vertex set of an outer tet and the matrix rows no longer fit in LDS, so the
integration and the row assembly keep their fixed-point sums in device
memory.  Checked against the oracle at delta = 7h on an outer subset, and
bitwise against the LDS form (forced global sums on a workload that fits)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import helpers as H
import meshgen as mg

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _say(msg):
    sys.stdout.write(f"[gpu-test] {msg}\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_07499_amd as P
    d = P.Device(0)
    yield d
    d.close()


@pytest.mark.parametrize("keying", ["pair", "element"])
def test_delta_7h_subset_vs_oracle(dev, orc, keying):
    import paper_2302_07499_amd as P
    pb = mg.make_problem("wide7", 20, delta_over_h=7.0, jitter=0.15, jitter_seed=71, mc_samples=16, seed=5)
    pb.keying = keying
    mask = mg.outer_subset_mask(pb.mesh.n_tets, 0.01, seed=17)
    _say(f"delta = 7h on 20^3 cubes, {int(mask.sum())} outer tets, keying {keying}")
    plan = dev.plan_problem(pb, outer_mask=mask)
    g = P.system_to_numpy(plan.assemble(pb.f_qp, pb.g_nodal))
    plan.destroy()
    _say("oracle ...")
    o = orc.problem_assemble(pb, outer_mask=mask)
    assert np.array_equal(g["pair_counts"], o["pair_counts"])
    H.pattern_equal(g, o)
    e = H.value_errors(g, o)
    _say(f"  errors {e}")
    assert e["ff_abs"] <= FP64_TOL and e["fc_abs"] <= FP64_TOL and e["rhs"] <= FP64_TOL


_FORCED = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
import meshgen as mg, paper_2302_07499_amd as P
dev = P.Device(0)
pb = mg.make_problem("fg", 9, delta_over_h=3.0, jitter=0.15, jitter_seed=5, mc_samples=16, seed=2)
pb.keying = {keying!r}
plan = dev.plan_problem(pb)
g = P.system_to_numpy(plan.assemble(pb.f_qp, pb.g_nodal))
np.savez({out!r}, ff=g["ff_val"], fc=g["fc_val"], rhs=g["rhs"])
plan.destroy(); dev.close()
"""


@pytest.mark.parametrize("keying", ["pair", "element"])
def test_global_sums_equal_lds_sums(tmp_path, keying):
    """The same plan with every sum forced into device memory gives bitwise the
    LDS results, in either keying."""
    res = {}
    for mode in ["0", "1"]:
        out = str(tmp_path / f"r{mode}.npz")
        env = dict(os.environ, NLFEM_GLOBAL_SUMS=mode)
        _say(f"forced global sums = {mode}, keying {keying}")
        r = subprocess.run([sys.executable, "-c", _FORCED.format(root=ROOT, keying=keying, out=out)], env=env,
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        res[mode] = np.load(out)
    a, b = res["0"], res["1"]
    for k in ["ff", "fc", "rhs"]:
        assert np.array_equal(a[k], b[k]), k
