"""MI355X-native hot path of QUEEN's per-frame residual fitting (differentiable 3D Gaussian splatting).

Importing the package loads nothing; ``paper_2412_04469_amd.qg`` loads the HIP library ``libqg.so`` and
raises if it is missing.
"""
__all__ = ["synth"]
