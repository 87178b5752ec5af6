"""The uneven batch replayed as one captured HIP graph (rrc_batch_run with
RRC_BATCH_GRAPH).  Kept out of collection until it has passed on the GPU."""
import numpy as np
import pytest
import torch

from tests.test_gpu_parity import DEV, _batch_inputs

pytestmark = pytest.mark.gpu


def test_batch_graph_matches_eager_runs(rrc):
    # the whole uneven batch captured once (fork/join over branch and
    # auxiliary streams) and replayed as one graph launch: every replay, with
    # eager work and synchronisation in between, equals the eager runs
    plans, volts, gins = _batch_inputs(rrc)
    ref = [p.run(v, gains_in=gi, mode="pipelined") for p, v, gi in zip(plans, volts, gins)]
    torch.cuda.synchronize()
    batch = rrc.Batch(plans, graph=True)
    outs = [p.alloc_outputs(DEV) for p in plans]
    for rep in range(4):
        for o in outs:
            for t in o.values():
                t.fill_(7)
        torch.cuda.synchronize()
        batch.run(volts, gins, outs, mode="pipelined")
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(outs, ref)):
            for key in ("vunique", "vauto", "vred", "gains", "vmodel", "chisq", "niter", "status"):
                assert torch.equal(o[key], r[key]), (rep, k, key)
    del batch
