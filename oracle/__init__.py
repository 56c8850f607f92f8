"""Plain CPU oracle for the two-site TDVP effective-Hamiltonian hot path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call,
link or execute anything in this package: only ``tests/``, the smoke check
in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` use it.

Everything here is deliberately plain and slow: dense complex128 numpy /
scipy arithmetic on full (Clebsch-Gordan expanded) tensors, written from the
paper's statement of the method and from textbook definitions, so that a
reader can check it against the paper by eye.  It shares no code, headers,
tables or constants with the HIP library; only the seeded input generators
in ``synth`` serve both sides.

Modules
-------
cg        Clebsch-Gordan coefficients from the Racah formula (exact rationals).
fermions  Jordan-Wigner fermions, the Hubbard Hamiltonian of the paper's
          Eq. (1) (and its particle-hole symmetric form), exact time
          evolution of a state vector, site observables.
reduced   Expansion of U(1)xSU(2) reduced tensors to full tensors under the
          documented Wigner-Eckart conventions.
dense     Dense MPS algebra: environments, the effective Hamiltonian as a
          plain definition, Lanczos / exact matrix exponentials and a
          symmetric second-order two-site TDVP sweep.
sampled   Sector-restricted evaluation of selected output blocks of the
          effective Hamiltonian and environment update, for sizes where the
          full dense problem does not fit.
"""
