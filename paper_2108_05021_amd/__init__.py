"""MI355X-native one-sided box filter (Gong, "One-Sided Box Filter for Edge
Preserving Image Smoothing", arXiv 2108.05021).

The filter runs in hand-written HIP kernels for gfx950 behind the C ABI in
``include/osbf.h``; :mod:`paper_2108_05021_amd.osbf` is the thin ctypes binding
(argument marshalling only) and :mod:`paper_2108_05021_amd.synth` draws the
seeded synthetic inputs.  Importing this package loads nothing; the HIP library
is loaded on first use and its absence is an error.
"""
__all__ = ["osbf", "synth"]
