"""MI355X-native constant-potential-method electrode charge solve.

The compute path lives in the HIP library `libcpm.so` (sources under
`csrc/`, C-ABI in `include/cpm.h`); `cpm` is its thin ctypes binding and
`inputs` builds seeded synthetic capacitors.  Importing the package loads
nothing: the library is opened on first use by `cpm.lib()`.
"""
