"""Two qualitative claims of the paper, reproduced by the FP64 oracle on seeded
synthetic damped-exponential series (information about the method, not parity
pins; the GPU path is checked against the oracle elsewhere):

* Sec. IV / Fig. 3: the GIRAF approximation, circular along the echoes, fits
  decaying signals worse than the hybrid lifting (linear along the echoes);
* Sec. IV / Table 1b: a filter with several taps along the echoes recovers the
  series better than a single tap (joint sparsity only).
"""
import numpy as np
import pytest

import oracle
import workload


@pytest.mark.parametrize("seed", [201, 202, 203])
def test_hybrid_lifting_beats_giraf_and_a_single_tap(seed):
    pb = workload.make_problem(seed=seed, P=32, Q=32, T=10, K=2, R=4, N1=5, N2=5, M=3, n_irls=8, n_cg=8)
    err = lambda x: np.linalg.norm(x - pb.truth) / np.linalg.norm(pb.truth)
    hybrid = err(oracle.irls(pb.b, pb.S, 5, 5, 3, pb.lam, 8, 8))
    giraf = err(oracle.irls(pb.b, pb.S, 5, 5, 3, pb.lam, 8, 8, circ_t=True))
    one_tap = err(oracle.irls(pb.b, pb.S, 5, 5, 1, pb.lam, 8, 8))
    assert hybrid < 0.9 * giraf, (hybrid, giraf)
    assert hybrid < 0.7 * one_tap, (hybrid, one_tap)
