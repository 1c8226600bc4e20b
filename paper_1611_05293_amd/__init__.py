"""MI355X-native VFP split step (arXiv:1611.05293) behind the C-ABI library
``libvfp.so``.  Importing the package loads nothing; ``paper_1611_05293_amd.vfp``
is the thin ctypes binding, ``paper_1611_05293_amd.inputs`` the seeded
synthetic input generators."""
