"""MI355X-native forward semi-Lagrangian advection (Becerra-Sagredo, Malaga &
Mandujano): trajectory integration of the material lattice and Z-spline
reconstruction on the reference mesh, as HIP kernels for gfx950 behind a C ABI.

``workloads`` (seeded inputs) imports without the GPU library; the binding in
``binding`` loads ``libsl.so`` on first use and fails loudly when it is
missing.
"""
