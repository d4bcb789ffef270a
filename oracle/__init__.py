"""CPU oracle for tensor-train Fourier pricing of multi-asset options.

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports, links or runs
anything in this directory; only the tests, the smoke check and the benchmark's
CPU-baseline leg do. The oracle shares no code with the GPU path.

Modules
    closed_forms  Black-Scholes (Eq. BSexact), bivariate normal, Stulz two-asset
                  max/min calls, Margrabe exchange value, one-factor quadrature for
                  max/min calls and puts at any d.
    fourier       the d-dimensional Fourier price on a truncated uniform grid
                  (Eq. maincont, Eq. main, Eq. discr and the nested sum of Sec. III.D),
                  decomposed into one separable term per asset for max/min payoffs,
                  summed densely by the plain C loop in dense.c.
    mc            exact-terminal Monte Carlo (Sec. III.A, Eq. mc).
    greeks        central finite-difference Greeks on the dense Fourier price.
    ttcross       a plain NumPy TT-cross (Sec. IV.B): matrix cross, maxvol, sweeps.
    mlp           a plain NumPy MLP (forward, backward, Adam) for the price surrogate.

Parity status of each function is stated in its module header.
"""
