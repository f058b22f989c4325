"""CPU oracle for the two-determinant DCSD / CCSD residual.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The product path (``paper_2401_11935_amd`` and ``libdcsd``) never calls it,
and the oracle never imports the product; the two share only the seeded
input generator ``dcsd_synth`` (which holds none of the method's arithmetic).

Everything here is plain NumPy in FP64, written from the paper's Theory
section:

* ``hamiltonian`` -- spin-orbital integrals and Fock matrices of the
  reference determinant Phi_A, built from DF factors B and a spin-averaged
  Fock matrix F (two singly occupied orbitals t, u; Fig. 1).
* ``ccsd``        -- the single-reference CCSD residual <x| e^-T H e^T |A>
  in explicit-T1 spin-orbital form (the connected term of the amplitude
  equations).
* ``dc``          -- the distinguishable-cluster modification: the T2*T2
  terms it drops from the doubles equations.
* ``coupling``    -- the coupling coefficient K_x = <A^x| e^-T_A e^T_B |B>
  with T_B the spin flip of T_A, evaluated exactly in the small Fock space
  each excitation lives in.
* ``twodet``      -- the 2D residual R_x = connected - dropped - K_x W, W,
  and the singlet/triplet energies Delta E_A +- W.
* ``solver``      -- Jacobi + DIIS iterations.
* ``brute``       -- a determinant-space engine (exact e^T, H, FCI) that
  pins the tensor code above on small systems.

Parity pinning status of each function is stated in its module header.
"""
