"""MI355X p-multigrid pressure Poisson solver (hybrid Fourier x Chebyshev, sigma-transformed)."""
