"""FP64 CPU oracle for hybrid SDC (HSDC) and two-level PFASST on the monodomain
equation (de Souza, Pezzuto, Krause, "High-order parallel-in-time method for
the monodomain equation in cardiac electrophysiology", arXiv 2405.19994).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
restatement of the method used to check the HIP library.  Only the test suite,
the smoke entry point and the CPU-baseline leg of the benchmark may import it;
the product path (the C-ABI library and its Python binding) never does, and the
two share no code.

Modules
-------
coeffs     Radau IIA nodes, Lagrange derivative weights, phi_k, a_ij(z), R/T
ttp06      ten Tusscher-Panfilov 2006 epicardial cell model (node-wise)
tissue     cell-centred no-flux Laplacian, direct solves, space transfer
problems   ODE problems y' = f_I + f_E + f_e (monodomain, scalar test)
hsdc       collocation operator C, preconditioner P, sweep, serial stepping
pfasst     Algorithm 1 (FAS over levels, Q^seq / Q^par, burn-in)

Parity status of every function is stated in its docstring ("pinned by ..."
or "parity unpinned").
"""
