"""CPU oracle for the QAOA-MaxCut energy path -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in this package.  The GPU library
(``paper_2106_15740_amd``) never imports it, and this package never imports
the library: the two share no code, only the seeded inputs of ``workloads``.

Contents (each function cites the passage of the paper it follows):

* ``statevector``  complex128 state-vector simulation of the QAOA ansatz
  (Section II, eq. qaoa1), the per-edge <Z_j Z_k>, the MaxCut energy
  E = <C> and its gradient by the adjoint-state method and by central finite
  differences.  This is the plain definition of what the tensor-network path
  computes.
* ``ball``         the same definition restricted to the radius-p ball around an
  edge (the light-cone argument of Section II), for graphs too large for a
  full state vector.
* ``tn``           an independent tensor-network contraction of one edge term:
  light cone by pruning a gate list, diagonal-gate network (Section IV.B),
  bucket elimination with numpy einsum (Section III.B).

Pins: every function here is checked in ``tests/test_oracle_pins.py`` against
results fixed by the mathematics (dense-matrix exponentials, the published
p=1 closed form, exact special values, symmetries) and not by this code.
"""
