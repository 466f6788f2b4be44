"""MI355X-native effective-resistance analysis for stacked 3D-IC power
delivery networks.

The compute path lives in ``libreff.so`` (HIP for gfx950 behind a C ABI);
``paper_2607_05818_amd.reff`` is its thin ctypes binding.  Importing the
package itself loads nothing, so the seeded input generators in
``paper_2607_05818_amd.gen`` can be used without a GPU.
"""
__all__ = ["gen", "reff"]
