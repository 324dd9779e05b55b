"""MI355X-native differentiable radar ambiguity function (GRAF hot path).

Importing the package loads nothing native; the HIP library is opened on
first use by ``paper_2506_22935_amd.af`` and fails loudly when it is missing.
"""
__all__ = ["af", "workloads"]
