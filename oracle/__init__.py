"""CPU complex128 oracle for sliced tensor-network contraction of random circuits.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU product path never
calls it and shares no code with it.

* ``contract``    -- pairwise path contraction with slicing (Sec. 2.4, 3.1, 3.2)
* ``naive``       -- explicit-loop contraction of tiny networks
* ``statevector`` -- brute-force state-vector simulation of the circuit
* ``metrics``     -- amplitude error measures (Sec. 4.3)
* ``split``       -- hi/lo operand splitting and split dot products of the
                     extended-precision products (Sec. 4.2)

Pinned by tests/test_oracle_pins.py against the state vector, closed forms,
normalisation, slicing and path invariance, and brute-force loops.
"""
