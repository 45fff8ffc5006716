"""MI355X-native parareal evaluation of matrix functions.

The compute path is the HIP library ``libfm.so`` (C ABI declared in
``include/fm.h``); ``paper_1505_07959_amd.fm`` is its thin ctypes binding.
``paper_1505_07959_amd.inputs`` holds the seeded synthetic workloads.
Importing the package loads nothing; importing ``fm`` loads the library and
fails loudly when it is missing.
"""
