"""MI355X (gfx950) engine for checkerboard Metropolis on the 3D +-J spin glass
with asynchronous multispin coding (Lulli, Bernaschi, Parisi, arXiv:1411.0127).

The compute path is the HIP library ``libsg.so`` behind the C ABI of
``include/sg.h``; ``paper_1411_0127_amd.sg`` is its Python binding.  Importing the
package itself loads nothing, so that the build step can run first.
"""

__all__ = ["sg"]
