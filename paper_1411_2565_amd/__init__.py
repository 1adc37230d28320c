"""MI355X-native micromagnetic step: FFT demag + exchange + anisotropy +
Zeeman effective field and explicit-Euler LLG update, as hand-written HIP
kernels for gfx950 behind a C ABI (``include/mm.h``).

Only ``binding`` touches the native library; ``workloads`` holds seeded
inputs.  Importing the package does not load the GPU library.
"""
