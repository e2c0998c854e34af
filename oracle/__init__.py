"""CPU FP64 oracle of the conic interior-point method of arXiv 2412.19027.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
benchmark's cpu_baseline leg may import anything from this package; the GPU
library and its Python binding never do, and the two share no code.

Modules:
  jets    -- truncated Taylor arithmetic for barrier derivatives
  cones   -- per-family cone operations (scalings, Jordan algebra, steps)
  linsys  -- block-elimination LDL' of the quasi-definite KKT system + IR
  ipm     -- setup (equilibration, initial point) and the Algorithm 1 loop
"""
