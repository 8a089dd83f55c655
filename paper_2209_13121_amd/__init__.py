"""MI355X-native fast multipole method for the 3-D Coulomb (Laplace) sum.

The compute path is the C-ABI library ``libfmm.so`` (hand-written HIP for
gfx950, declared in ``include/fmm.h``); ``binding`` marshals torch tensors into
it.  Nothing is imported eagerly so that ``workloads`` stays usable on hosts
without the built library.
"""
__all__ = ["binding", "workloads"]
