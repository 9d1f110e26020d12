"""Call-auction ensemble engine for AMD Instinct MI355X (gfx950).

Submodules:
  engine     -- ``Ensemble`` (create / step / read books and statistics) over libcae's C ABI
  workloads  -- seeded synthetic market descriptors for the benchmark shapes
  build      -- hipcc build of libcae.so

Importing the package does not load the GPU library; ``engine`` does, and fails loudly if it
has not been built.
"""
__all__ = ["engine", "workloads", "build"]
