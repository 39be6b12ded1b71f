"""fewbody on MI355X: FP64 time-symmetrised Hermite P(EC)^2 integration of very
many independent few-body planetary systems (the method of Swarm-NG,
arXiv:1208.1157, Section 2.2.1 and Algorithm 2), as hand-written HIP kernels
for gfx950 behind a C ABI (``include/fewbody.h``).

Submodules:
  gen      -- seeded synthetic ensembles and the serving request trace
  fewbody  -- ctypes binding of libfewbody.so (loads the HIP library; raises
              if it is missing)
  autotune -- per-body-count launch-plan search over the library's plans
  serve    -- Poisson-trace driver of the library's continuous-batching server
"""
