"""Plain FP64 CPU oracle for the stabilized space-time IgA solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports it and
shares no code with it.

Everything here follows the paper's definitions literally and slowly:
univariate B-splines by the Cox-de Boor recursion (Section 2), Galerkin forms
evaluated by Gauss quadrature and assembled into explicit sparse space-time
matrices (Section 3, the forms A, S, L and the matrices of Section 3.1.1),
the SU activation theta of eq. (3.6) with support extensions (eq. (2.3)), its
truncated-SVD low-rank approximation (eq. (3.9)), the w-update of Section 3.2,
and direct sparse solves (scipy ``splu``).

Readings of points where the paper is silent or ambiguous are listed in the
module docstrings where they are used.
"""
