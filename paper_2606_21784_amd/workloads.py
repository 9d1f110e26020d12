"""Seeded synthetic workloads (market descriptors, generator seed, step count).

This module draws inputs only; it holds none of the engine's arithmetic.  The shapes follow the
paper's sweeps (section IV: M markets x A zero-intelligence agents x L ticks x S steps) at the
sizes this project benchmarks.  Descriptor draws for the uneven ensemble and the calibration
parameters use numpy's PCG64 generator with fixed seeds.
"""
import numpy as np

MARKET_DTYPE = np.dtype([
    ("L", np.uint32), ("A", np.uint32), ("K", np.uint32), ("Q", np.uint32),
    ("n_noise", np.uint32), ("n_mom", np.uint32), ("h", np.uint32), ("flags", np.uint32),
])


def uniform(M, L, A, K, Q, n_noise=None, n_mom=0, h=2, flags=0):
    d = np.zeros(M, MARKET_DTYPE)
    d["L"], d["A"], d["K"], d["Q"] = L, A, K, Q
    d["n_noise"] = A if n_noise is None else n_noise
    d["n_mom"], d["h"], d["flags"] = n_mom, h, flags
    return d


def smoke():
    """4 markets, L=64, A=128 noise agents, offsets +-8, qty 1..10, 100 steps, seed 0."""
    return {"name": "smoke_M4_L64_A128_S100", "descs": uniform(4, 64, 128, 8, 10),
            "seed": 0, "S": 100}


def fixed():
    """The fixed standard workload: 1024 markets, L=256, A=1024, offsets +-16, qty 1..100,
    1000 steps, seed 1 (1.049e9 agent events, the paper's fixed-workload event count)."""
    return {"name": "fixed_M1024_L256_A1024_S1000", "descs": uniform(1024, 256, 1024, 16, 100),
            "seed": 1, "S": 1000}


def paper_fixed():
    """The paper's fixed-workload shape (section IV-E, Table IV): 8192 markets, A = 256,
    L = 128, 500 steps (1.049e9 events).  Offsets +-8 and quantities 1..10 (the paper does not
    state its values), seed 2."""
    return {"name": "paperfixed_M8192_L128_A256_S500", "descs": uniform(8192, 128, 256, 8, 10),
            "seed": 2, "S": 500}


def paper_market_sweep(M):
    """The paper's market-count sweep shape (section IV-E, Table III top): A = 256, L = 128,
    500 steps; offsets +-8 and quantities 1..10, seed 2."""
    return {"name": "papersweep_M%d_L128_A256_S500" % M, "descs": uniform(M, 128, 256, 8, 10),
            "seed": 2, "S": 500}


def paper_agent_sweep(A):
    """The paper's agent-count sweep shape (section IV-E, Table III bottom): 8192 markets,
    L = 128, 500 steps; offsets +-8 and quantities 1..10, seed 2."""
    return {"name": "paperagents_M8192_L128_A%d_S500" % A, "descs": uniform(8192, 128, A, 8, 10),
            "seed": 2, "S": 500}


PAPER_SWEEP_M = (64, 256, 1024, 4096, 16384)
PAPER_SWEEP_A = (16, 64, 256, 1024)


def market_sweep(M):
    """Market-count sweep point: L=512, A=4096, offsets +-32, qty 1..100, 10000 steps, seed 3."""
    return {"name": "sweep_M%d_L512_A4096_S10000" % M, "descs": uniform(M, 512, 4096, 32, 100),
            "seed": 3, "S": 10000}


MARKET_SWEEP_M = (16, 64, 256, 1024, 4096, 16384, 65536)


def uneven(M=8192, seed=4):
    """Uneven ensemble: L uniform on {64,...,1024}, A log-uniform on [64, 16384], K = L/16,
    qty 1..100, 2000 steps, generator seed 4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.array([64, 128, 256, 512, 1024])[rng.integers(0, 5, M)]
    A = np.rint(np.exp(rng.uniform(np.log(64.0), np.log(16384.0), M))).astype(np.int64)
    A = np.clip(A, 64, 16384)
    d = np.zeros(M, MARKET_DTYPE)
    d["L"], d["A"], d["K"], d["Q"] = L, A, L // 16, 100
    d["n_noise"], d["n_mom"], d["h"] = A, 0, 2
    return {"name": "uneven_M%d_S2000" % M, "descs": d, "seed": 4, "S": 2000}


# Calibration parameters: noise fraction U[0,1], momentum fraction U[0, 1-noise], offset width
# U[2,32] ticks, mean quantity U[5,100]; each draw is an ensemble of 64 markets at L=256,
# A=1024 and 2000 steps.  Quantities are uniform on {1..Q} with Q = round(2*mean - 1) so that
# their mean is the drawn mean; makers post 2 ticks from the reference.
CALIB_L, CALIB_A, CALIB_S, CALIB_MARKETS, CALIB_H, CALIB_SEED = 256, 1024, 2000, 64, 2, 5


def calibration_params(n=65536, seed=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    f_noise = rng.uniform(0.0, 1.0, n)
    f_mom = rng.uniform(0.0, 1.0, n) * (1.0 - f_noise)
    width = rng.uniform(2.0, 32.0, n)
    mean_q = rng.uniform(5.0, 100.0, n)
    return np.stack([f_noise, f_mom, width, mean_q], axis=1)


def calibration_markets(theta, first_draw=0, markets_per_draw=CALIB_MARKETS):
    """Descriptors of the ensembles of parameter rows theta[i] (draw index first_draw + i).
    Market index of draw j, replica r is j * markets_per_draw + r within the returned array."""
    theta = np.atleast_2d(theta)
    n = len(theta)
    A = CALIB_A
    n_noise = np.rint(theta[:, 0] * A).astype(np.int64)
    n_mom = np.minimum(A - n_noise, np.rint(theta[:, 1] * A).astype(np.int64))
    K = np.rint(theta[:, 2]).astype(np.int64)
    Q = np.rint(2.0 * theta[:, 3] - 1.0).astype(np.int64)
    d = np.zeros(n * markets_per_draw, MARKET_DTYPE)
    rep = lambda x: np.repeat(x, markets_per_draw)
    d["L"], d["A"] = CALIB_L, A
    d["K"], d["Q"] = rep(K), rep(Q)
    d["n_noise"], d["n_mom"], d["h"] = rep(n_noise), rep(n_mom), CALIB_H
    return d


def test_split(n):
    """Indices of the held-out 10% (every draw with index % 10 == 9) and the training 90%."""
    idx = np.arange(n)
    return idx[idx % 10 != 9], idx[idx % 10 == 9]
