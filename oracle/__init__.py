"""CPU FP64 oracle for the APF scattering matrix and its permittivity gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the library may import, call or link
anything in this package; only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path:
it assembles its own operator, solves with its own block LU, and forms S and
the gradient from the plain definitions:

* S = C A^-1 B - D  (Sec. 2, the generalised scattering matrix),
* df/deps_k = sum_nm 2 Re(dF/dS_nm dS_nm/deps_k)  (Eq. 1),
* dS/deps_k = -(C A^-1 u_k) sigma_k (u_k^T A^-1 B)  (Eqs. 2-3 with u_k = e_k).

Modules:
    fdfd       discretised operator A, source matrix B, projection matrix C
    blocksolve block-tridiagonal LU in y-row blocks, cyclic block LU in x-columns
    apf        S, objective, weighted-adjoint gradient and the cross-check routes
"""
