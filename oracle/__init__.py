"""FP64 CPU oracle for HoloGen-style hologram generation.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously
correct statement of what the GPU hot path computes, written from the
HoloGen paper (Christopher et al., "HoloGen: An open-source toolbox for
high-speed hologram generation", arXiv 2008.12214).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import it.  The product path (``paper_2008_12214_amd``) never imports,
links or calls anything here, and this package imports nothing from the
product path.  The two share no code; only the seeded input generators in
``synth`` feed both sides.

Everything is float64 / complex128 on the CPU.  Discrete Fourier transforms
are written out as DFT-matrix products (the plain definition, Background
section, Eqs. fouriertrans2d5c/d); no FFT is used on the oracle side.

Modules
-------
dft       the unitary 2D DFT pair, centring of the replay plane
philox    Philox4x64-10 counter-based generator (Salmon et al., SC'11)
slm       SLM constraint: projection onto continuous or L-level phase
metrics   MSE (Error Metrics section, Eq. mse) and scale-optimal NMSE
hologram  target preparation, Fresnel chirp, GS, weighted GS, OSPR
search    direct search and exhaustive search on tiny grids
nn        learned-initialisation network layers (forward/backward, FP64)

Functions whose result is not pinned by an independent check say
"parity unpinned" in their docstring.
"""
