"""Call-auction ensemble engine for AMD Instinct MI355X (gfx950).

Submodules:
  engine     -- ``Ensemble`` (create / step / traced step / read books and statistics) over
                libcae's C ABI
  workloads  -- seeded synthetic market descriptors for the benchmark shapes
  autotune   -- per-size-class schedule search for uneven ensembles
  dynamics   -- agent-mix sweeps and stylized facts from traced price and volume series
  mlp        -- the calibration surrogate's bf16 MLP (forward, backward, Adam) over the C ABI
  surrogate  -- data generation, training and judging of the surrogate
  build      -- hipcc build of libcae.so

Importing the package does not load the GPU library; ``engine`` does, and fails loudly if it
has not been built.
"""
__all__ = ["engine", "workloads", "autotune", "dynamics", "mlp", "surrogate", "build"]
