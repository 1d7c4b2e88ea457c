"""Host logic of the Python binding that needs no GPU: the checkpointed
run's accumulator carving (several zeroed states as views of one buffer)."""
import math

import pytest
import torch

from paper_2506_04857_amd import inputs as I

af = pytest.importorskip("paper_2506_04857_amd.af_mhd")


def carved(prob, n):
    run = af.CheckpointedRun.__new__(af.CheckpointedRun)
    run.prob = prob
    run.device = torch.device("cpu")
    return run._zero_states(n)


@pytest.mark.parametrize("bc", [I.PERIODIC, I.OUTFLOW])
def test_zero_states_are_disjoint_contiguous_zero_views(bc):
    prob = I.random_smooth(7, 5, seed=1, bc=bc)
    states = carved(prob, 3)
    assert len(states) == 3
    total = sum(math.prod(s) for s in prob.shapes())
    spans = []
    for st in states:
        assert tuple(t.shape for t in st) == tuple(prob.shapes())
        for t in st:
            assert t.dtype == torch.float64 and t.is_contiguous()
            assert torch.count_nonzero(t) == 0
            spans.append((t.data_ptr(), t.data_ptr() + t.numel() * 8))
    spans.sort()
    # back to back, no overlap, covering exactly 3 states
    for (a0, a1), (b0, _) in zip(spans, spans[1:]):
        assert a1 == b0
    assert spans[-1][1] - spans[0][0] == 3 * total * 8
    # writing one view leaves the others zero
    states[1][2].fill_(1.0)
    assert torch.count_nonzero(states[0][2]) == 0 and torch.count_nonzero(states[2][2]) == 0
    assert torch.count_nonzero(states[1][3]) == 0
