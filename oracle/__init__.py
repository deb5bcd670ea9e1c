"""Plain FP64 CPU oracle for the local-energy path (test infrastructure only).

This package is the checker the HIP library is compared against. It is slow on
purpose and written to be read against the paper: every function states the
passage it follows. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never does.
It shares no code with the HIP library (not even the bitstring packing).

Modules
-------
``fock``           explicit creation/annihilation-operator Hamiltonian on a set of
                   determinants (Methods: second-quantised Hamiltonian and the
                   Jordan--Wigner map).
``slater_condon``  canonical list of the determinants connected to one determinant
                   and the matrix elements (Results, GPU-supported local energy:
                   the sum over coupled configurations; Methods: Hamiltonian).
``made``           the autoregressive amplitude/phase ansatz with the number-
                   conserving conditionals (Results: wavefunction ansatz, parallel
                   sampling), its hand-derived backward and an ancestral sampler.
``energy``         local energies, weighted energy statistics and the VMC gradient
                   (Results: local-energy sum; Methods: VMC objective, gradient
                   estimator, batch energy estimator).
``bf16``           FP64 -> FP32 -> BF16 round-to-nearest-even of parameters.
``pauli``          the paper's own route: Jordan--Wigner Pauli strings and their
                   matrix elements (Algorithm 1 and the Pauli-element equation), used
                   as an independent cross-check of the local energy.

Every function is pinned by a ``-m "not gpu"`` test in ``tests/test_oracle_pins.py``
against closed forms, invariants or brute force.
"""
