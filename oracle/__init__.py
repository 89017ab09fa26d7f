"""Plain FP64 CPU oracle for the even-odd Wilson operator (test infrastructure).

This package is test infrastructure only.  It is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``,
never by the library in ``paper_2303_08609_amd``; the two share no code.  It
works on the full lattice with explicit parity masks, full 4x4 gamma matrices
and full 3x3 links: no spin projection, no link compression and no even-odd
compaction inside the operator.  Everything is complex128.

Modules:

* ``gamma``      -- Euclidean Dirac matrices (paper Sec. 2 states only their
                    properties; the representation is a documented choice).
* ``lattice``    -- parity, coordinates and the even/odd compaction of
                    paper Sec. 3.3 (Fig. 4).
* ``wilson``     -- hopping term and Wilson matrix, Eq. (1) and its footnote;
                    even-odd blocks and the Schur operator, Eqs. (3)-(5);
                    a dense assembly from the footnote's component formula;
                    per-site evaluation for sampled checks on big lattices.
* ``solvers``    -- textbook CGLS, CG on the normal operator, FP64 defect
                    correction, dense solves (the paper names no solver).
* ``force``      -- derivatives of Re<eta, M psi> and <phi, (M^dag M)^-1 phi>
                    with respect to the spinors and the links.
* ``accounting`` -- flop and byte model of the operator (paper Sec. 2).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, a dense second route or central finite
differences; none is "parity unpinned".
"""
