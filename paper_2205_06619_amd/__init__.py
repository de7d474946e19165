"""FastSTMF on AMD MI355X (gfx950): sparse tropical matrix factorization.

Submodules:
  stmf   -- binding of the C ABI (include/stmf.h) over libstmf.so; importing it
            loads the HIP library and raises if it is missing
  synth  -- seeded synthetic inputs
  serve  -- continuous-batching serving loop over the engine entry points
  build  -- compiles csrc/*.hip into libstmf.so
"""

__all__ = ["stmf", "synth", "serve", "build"]
