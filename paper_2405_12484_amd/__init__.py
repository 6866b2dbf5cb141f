"""MI355X-native projective dynamics for volumetric homogenization.

The simulation runs in ``libvhpd.so`` (HIP kernels for gfx950 plus a native
C++ prefactor) behind the C ABI of ``include/vhpd.h``; ``vhpd`` is its Python
binding.  Importing this package does not load the library; ``vhpd.load()``
does, and raises when it has not been built.
"""
