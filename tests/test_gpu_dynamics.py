"""The composition sweep of the paper's section IV-J on the GPU: one traced launch over every
agent mix and population size; its series equal the oracle's and so do the statistics."""
import numpy as np
import pytest

import oracle as O
from paper_2606_21784_amd import dynamics

pytestmark = pytest.mark.gpu


def test_sweep_series_and_stats_match_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    A_values, alphas, markets, S = (16, 256), (0.0, 0.15, 0.7), 4, 200
    report, timing = dynamics.run_sweep(A_values=A_values, alphas=alphas, markets=markets, S=S)
    d = np.concatenate([dynamics.composition_descs(A, markets=markets, alphas=alphas)
                        for A in A_values])
    st, bk, pr, vo = O.run(d, 6, S, trace=True)
    ref = dynamics.series_stats(torch.from_numpy(pr.astype(np.int64)),
                                torch.from_numpy(vo.astype(np.int64)), 128,
                                torch.full((len(d),), 64), groups=len(A_values) * len(alphas))
    for j, A in enumerate(A_values):
        for k, v in ref.items():
            got = np.array(report[A][k], dtype=np.float64)
            want = v[j * len(alphas):(j + 1) * len(alphas)].numpy()
            np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-12, err_msg="%d %s" % (A, k))
    assert timing["events"] == float(d["A"].astype(np.float64).sum()) * S
    f = dynamics.facts(report, A=256, standard_alpha=0.15)
    assert isinstance(f["volatility_increases"], bool)
