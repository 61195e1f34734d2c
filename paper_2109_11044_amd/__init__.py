"""MI355X-native circulant-embedding conditional simulation with local
Kriging (Bailey, Bandyopadhyay and Nychka, arXiv 2109.11044).

The compute path is the HIP library ``libcesim.so`` (C ABI, ``include/cesim.h``);
``paper_2109_11044_amd.cesim`` is its thin ctypes binding.  Importing this
package loads nothing; the binding loads the library on first use and raises
if it has not been built.
"""

__all__ = ["cesim", "workloads"]
