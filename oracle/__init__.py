"""CPU oracle for the Ozaki-II emulated GEMM (accurate mode).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package; only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code,
tables or constant generators with the HIP library.

Contents
  constants  per-N constants of Section 3.1 (exact big integers, mpmath)
  fp         exact IEEE rounding helpers (Fractions; RN/RD/RU to FP32/FP64)
  ozaki2     Algorithms 1-3 step by step (scaling, residues, integer GEMMs,
             CRT reconstruction, inverse scaling)
  bounds     Theorem 1 (eq. thm:err-1), its simplified form (eq. thm:err-2)
             and the required-moduli reading of the planner
  exact      exact reference products (Fractions / Dekker + fsum)
  moduli     per-N moduli of largest product (Section 3.1), branch and bound
  complex_gemm  complex products on the real embedding (reading R23)
  twin       loader of os_ii_twin.cpp, a plain C++ (OpenMP) second
             implementation of Algorithms 1-3, compared stage by stage with
             ozaki2 and timed on every host core

Every floating-point step is either exact by a stated argument (and asserted),
or emulated with exact rational arithmetic followed by one correct rounding.
"""
