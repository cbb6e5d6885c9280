"""MI355X-native semi-stochastic local energy for BDG-RNN / MPS-RNN x cos-RBM
amplitudes (arXiv:2507.19276, Sec. 2.2-2.4).

Importing the package loads nothing; the HIP library is loaded on first use by
``paper_2507_19276_amd.nqs`` and raises if it has not been built.
"""
__all__ = ["workloads", "nqs"]
