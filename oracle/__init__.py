"""FP64 CPU oracle for GOFMM's evaluation phase (test infrastructure only).

This package is the checker, not the product.  Only the test suite, the
smoke check of the package entry and the CPU-baseline leg of the benchmark
may import it; the library never does, and it shares no code, header, table
or helper with the library.  Everything here is plain NumPy/SciPy in FP64,
written from the paper (Yu, Levitt, Reiz, Biros, "Geometry-Oblivious FMM for
Compressing Dense SPD Matrices", SC'17):

  kernels   K(I, J) entries of the synthetic kernels (the only input, Sec. 1
            "Problem statement").
  dense     exact K.W and the relative error eps_2 of Sec. 3.
  compress  a plain compression: Gram distances (Sec. 2.1, eqs. 3-4),
            metricSplit ball tree (Alg. 1), exact kappa-NN, LeafNear with the
            budget ballot (Alg. 2, eq. budget), FindFar (Alg. 3), MergeFar
            (Alg. 4), a symmetric refinement of the far pairs, nested
            interpolative decompositions (eqs. 7-8, Alg. 5).
  evaluate  the tree walk of Alg. 6 (N2S, S2S, S2N, L2L) and the dense
            assembly of K~ from the telescoped interpolation matrices.
  cfile     reader and writer of the compression file format exchanged with
            the library.

Parity status of every function is listed in its module header.
"""
