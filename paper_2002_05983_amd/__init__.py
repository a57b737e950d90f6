"""MI355X-native repeated star-stencil sweeps (2D/3D, radius 1-4).

The compute path lives in a C-ABI shared library built from csrc/ for gfx950;
``paper_2002_05983_amd.stencil`` is its thin Python binding.  Importing this
package does not load the library; the binding does, on first use.
"""
