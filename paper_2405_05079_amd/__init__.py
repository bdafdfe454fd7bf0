"""PoVar (Power Variable Projection) hot path on AMD Instinct MI355X (gfx950).

The compute path is the HIP library ``libpovar.so`` behind the C ABI declared
in ``include/povar.h``; ``paper_2405_05079_amd.povar`` is its ctypes binding.
It covers the three stages of the stratified pipeline: PoVar on the pOSE
objective, the projective refinement (RiPoBA on the reprojection objective)
and the metric upgrade with known intrinsics.
``paper_2405_05079_amd.synth`` draws seeded synthetic problems.  Importing the
package loads nothing; the binding loads the library on first use and raises
if it has not been built.
"""

__all__ = ["povar", "synth"]
