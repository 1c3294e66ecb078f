"""Plain FP64 CPU oracle for the multigrid path of the fourth-order AMR
projection method (Zhao & Zhang, arXiv 2506.02663).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP library (no kernels, headers, tables or helpers); the only thing the
two sides share is the seeded input generator module, which holds none of
the method's arithmetic.

Every function states the passage of the paper it follows.  The oracle
computes on dense per-level arrays (one array over the whole index space of
a level, with a cell mask), which is a different data model from the
packed per-box buffers of the HIP library.

Modules:
  fv     -- stencils and ghost-fill formulas of Section 3
  level  -- one refinement level: mask, ghost fill, operator, diagonal
  mg     -- the geometric multigrid of Section 6.5 and the outer loop
  amr    -- composite (multi-level) operators of Section 5.2-5.3
"""
