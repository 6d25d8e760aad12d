"""MI355X-native emulated-FP64 (Ozaki scheme) GEMM, two-site H_eff.psi and
Davidson solver.

``paper_2510_04795_amd.ozaki`` is the binding of the HIP library libozaki.so
(it raises ImportError when the library is not built);
``paper_2510_04795_amd.workloads`` holds the seeded synthetic inputs.  The
binding is imported lazily so the input generators never load the library.
"""


def __getattr__(name):
    if name == "ozaki":
        import importlib
        return importlib.import_module(".ozaki", __name__)
    raise AttributeError(name)
