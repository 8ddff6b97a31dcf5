"""Plain, slow, obviously correct FP64 CPU oracle for moment-conserving GW.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path;
the only common module is the seeded input generator ``gwsynth``, which
holds none of the method's arithmetic.

Modules
-------
gw          density-response moments (TDA and RPA), self-energy moments,
            block Lanczos from moments, upfolded Hamiltonian, QP assignment.
quadrature  the mapped Gauss-Legendre grid used for the RPA zeroth moment.
brute       brute-force references: full TDA/RPA diagonalisation, exact
            Lehmann self-energy moments and the exact upfolded Hamiltonian.
fsgw        the Fock / chemical-potential self-consistent loop (Alg. 2).
evgw        the eigenvalue self-consistent loop (App. A, Alg. A1).
qsgw        the quasiparticle self-consistent loop (Sec. 3.3, App. A Alg. A2).
naf         natural auxiliary functions (Sec. 2.1, eq. NAF).
spectral    spectral function, Aufbau filling, Dyson orbitals and the
            electron-number shift of a one-shot calculation (eqs. ret_GF,
            spectrum, density; Sec. 3.5).
mlp         the per-orbital MLP of the learned warm start (forward,
            gradient, Adam) in FP64.
"""
