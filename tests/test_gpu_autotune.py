"""GPU: the autotuner picks a feasible configuration, caches it per network
bucket, and the tuned options still give oracle-parity results."""
import json

import numpy as np
import pytest

import oracle
from paper_2503_18356_amd import inputs
from paper_2503_18356_amd import racipe as rp
from tests import parity

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def test_autotune_choose_cache_and_parity(tmp_path):
    from paper_2503_18356_amd.autotune import Autotuner, bucket
    topo = inputs.erdos_renyi(10, 25, 1002)
    path = str(tmp_path / "tune.json")
    tu = Autotuner(path)
    c = tu.tune(topo, rp.FP32, n_sets=500, n_ic=10, reps=1)
    T = rp.Topology.from_inputs(topo)
    assert T.lanes_supported(c.lanes) and c.refill_min >= 1 and c.solves_per_s > 0
    data = json.load(open(path))
    key = [k for k in data if bucket(T) in k][0]
    assert len(data[key]["all"]) >= 4
    # A second tuner reads the cache instead of measuring.
    c2 = Autotuner(path).tune(topo, rp.FP32, n_sets=1, n_ic=1)
    assert (c2.lanes, c2.refill_min) == (c.lanes, c.refill_min)
    # Tuned options keep parity with the oracle.
    opts = tu.opts(topo, rp.FP32)
    hp = rp.sample_params(T, 9, 100, 5)
    out = rp.steady_states(T, hp.to_device(), opts)
    torch.cuda.synchronize()
    net = oracle.canonicalize(topo.n_genes, topo.src, topo.dst, topo.sign)
    op = oracle.sample(net, 9, 100, 5)
    oo = oracle.Opts(ss_rtol=1e-5)
    ref = oracle.steady_states(net, op, oo, n_threads=8)
    rep = parity.compare_steady(net, op, oo, np.arange(500), out.x.cpu().numpy(), ref.x, 5,
                                out.status.cpu().numpy(), ref.status)
    assert rep.ok(), rep
