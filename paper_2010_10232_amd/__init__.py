"""MI355X-native deflated, multigrid-approximated CSLP + FGMRES solver for B-spline
(isogeometric) Helmholtz discretisations.

The compute path is the HIP library `libhh.so` (built from `csrc/`) behind the
C ABI declared in `include/hh.h`; `binding` marshals arguments to it with
ctypes.  The binding is imported lazily so that the input generators in
`workloads` can be used without loading the library.
"""


def __getattr__(name):
    if name == "binding":
        import importlib
        return importlib.import_module(__name__ + ".binding")
    raise AttributeError(name)
