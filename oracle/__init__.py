"""Plain FP64 CPU oracle of the SLIM system matrix-vector product.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything under this package;
only tests, the smoke check and the CPU-baseline leg of the benchmark do.

The oracle is written from the paper (Marek, Sharma, Triverio, "A Parallel
Boundary Element Method for the Electromagnetic Analysis of Large Structures
With Lossy Conductors") and shares no code with the GPU library.  Every
function names the passage it follows.  Modules:

    rwg        mesh checks, RWG basis, sparse D, B, F, I_x (Sec. II, eq. (2)-(3))
    quad       triangle quadrature, singular polar rule, pair integrals
    operators  dense L_A, L_phi, interior L, K, Z (4), Y_eq (5), M = Y_eq Z (6),
               and the system product of (7)-(8)
    aim        AIM decomposition (11): stencils P, grid convolution H, W = P^T,
               precorrected near field L_NR
    solve      dense LU solve, FP64 GMRES and flexible GMRES of (7)
    mgf        reflected multilayered-medium Green's functions (Sommerfeld integrals, TL model)
    precond    conductor-block (block Jacobi / restricted additive Schwarz) preconditioner
    sched      LPT (Alg. 1, bound (13)), modified Part_Schedule (Alg. 2, (14))
    mlp        FP64 reference of the scheduler's cost-model network
"""
