"""The paper's approximation study (Sec. IV, Figs. 2 and 3), reproduced by the FP64
oracle on seeded synthetic damped-exponential series (information about the
method, not parity pins; the GPU path is checked against the oracle elsewhere):

* Fig. 3: the GIRAF approximation, circular along the echoes, fits decaying
  signals worse than the hybrid lifting (linear along the echoes);
* Figs. 2 and 3: the hybrid lifting's FFT-based approximations reach the quality of
  IRLS-direct (the explicit lifting, linear in all three dimensions), and the two
  solutions are close to each other.
"""
import numpy as np
import pytest

import oracle
import workload


@pytest.mark.parametrize("seed", [201, 202, 203])
def test_hybrid_lifting_beats_giraf_and_matches_irls_direct(seed):
    pb = workload.make_problem(seed=seed, P=32, Q=32, T=10, K=2, R=4, N1=5, N2=5, M=3, n_irls=8, n_cg=8)
    err = lambda x: np.linalg.norm(x - pb.truth) / np.linalg.norm(pb.truth)
    x_hybrid = oracle.irls(pb.b, pb.S, 5, 5, 3, pb.lam, 8, 8)
    x_direct = oracle.irls_direct(pb.b, pb.S, 5, 5, 3, pb.lam, 8, 8)
    hybrid, direct = err(x_hybrid), err(x_direct)
    giraf = err(oracle.irls(pb.b, pb.S, 5, 5, 3, pb.lam, 8, 8, circ_t=True))
    assert hybrid < 0.9 * giraf, (hybrid, giraf)
    assert abs(hybrid - direct) < 0.1 * direct, (hybrid, direct)
    assert np.linalg.norm(x_hybrid - x_direct) < 0.5 * np.linalg.norm(x_direct - pb.truth)
