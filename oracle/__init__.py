"""Independent FP64 CPU oracle for the sparsifying-preconditioned Maxwell solve.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check and
the benchmark's CPU-baseline leg may import or run anything in this package.
The GPU library never calls it, and it shares no code with the GPU path:
every function here is written directly from the paper (Liu & Ying,
"Sparsifying preconditioner for the time-harmonic Maxwell's equations") in
plain NumPy / SciPy double precision, one step at a time in the paper's
order and notation, so that it can be read against the paper by eye.

Modules
  kernel   : grid and the dyadic Green's tensor K = (k^2 I + grad grad) G
  operator : dense and FFT Nystrom apply of A = I + K diag(m), the right-hand
             side, and the FFT symbol of the circulant embedding
  stencil  : neighbourhoods, the 27 position classes, the SVD stencil fit
             (alpha, beta), the medium-weighted per-point fit and its gauge
  sparse   : assembly of the sparse rows S and Q and the preconditioner S^-1 Q
  fgmres   : right-preconditioned flexible GMRES in FP64
  mlp      : the small stencil-prediction network (forward, backward, Adam)

Parity status of every function is listed in each module's header.
"""
