"""MI355X-native quantum-kernel Gram engine (exact MPS, HIP for gfx950).

Importing the package does not load the HIP library; the binding in
``qsvm`` loads ``libqsvm.so`` on first use and raises if it is missing.
"""

__all__ = ["qsvm", "synth"]
