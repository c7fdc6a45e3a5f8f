"""Mandelbrot dwell images on MI355X (gfx950) by exhaustive evaluation and by
Mariani-Silver subdivision as Adaptive Serial Kernels and as a persistent
queue kernel (arXiv 2206.02255).

The work runs in ``libask.so`` (HIP, C ABI in ``include/ask.h``); ``ask`` is
its Python binding.
"""
