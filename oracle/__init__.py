"""FP64 CPU oracle for the transcorrelated (TC / BITC) operator of arXiv:2302.07420.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (no kernels, tables, constants or helpers); both sides consume the
same seeded inputs from ``tcinputs``.

Modules
  fftroute  the operator evaluated term by term following the paper's
            algorithms (Secs. 2.6.3-2.6.4, Algs. 2ah/2ax/3a1-3a4/3b1-3b6) with the
            Gygi-Baldereschi corrections (Sec. 2.5 and the per-term equations),
            the pseudo-energy (Eqs. EtotTC / EtotBiTC) and its autograd gradient.
  brute     the same discrete quantities as literal real-space double and triple
            sums over all permutations of the determinant (Sec. 2.6 notation).
  heg       closed forms for plane-wave (electron gas) orbitals: every term is
            diagonal and reduces to finite sums over occupied momenta.

Parity status of each function is stated in its docstring; every function here
is pinned by a ``-m "not gpu"`` test (see tests/test_oracle_*.py) except where a
docstring says "parity unpinned".
"""
