"""MI355X-native K_nu(x) by finite-window quadrature of its integral form, and
tiled Matern covariance generation built on it (arXiv 2502.00356, Sec. IV).

The compute path is the HIP library libbesselk.so (C ABI, include/besselk.h);
`paper_2502_00356_amd.api` is its ctypes binding. `workloads` holds the seeded
input generators.
"""
