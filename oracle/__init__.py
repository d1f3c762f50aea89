"""Plain CPU oracle for the CROSS hot path (arXiv 2501.07047).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, headers,
tables or constants with the HIP library under ``paper_2501_07047_amd/``.

Every function is written for obviousness, not speed: plain definitions in
Python integers or NumPy ``uint64`` (28-bit residues, so every product of two
residues is below 2**56 and exact).  Each function cites the passage of the
paper it follows (section / equation / algorithm / table).

Modules
  primes     -- NTT-friendly prime chain, Miller-Rabin, generator, psi
  ntt        -- negacyclic NTT by definition (O(N^2)), textbook CT/GS NTT
  poly       -- schoolbook negacyclic product
  mat        -- the layout-invariant 3-step NTT (Sec. MAT) in matrix form
  bat        -- BAT chunk decomposition / ModMatMul model (Alg. bat_deployment)
  reduction  -- Montgomery (Alg. montgomery_reduction) and Barrett (Alg. barrett)
  bconv      -- fast basis conversion (App. BConv), big-integer and uint64
  ckks       -- hybrid key switching, HE-Mult, automorphism, rotation
"""
