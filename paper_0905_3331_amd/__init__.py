"""MI355X (gfx950) twisted-mass Dirac operator and CG solver.

The even/odd preconditioned Wilson twisted-mass operator and the CG solve of
Qhat^+ Qhat^- x = b (Jansen & Urbach, "tmLQCD", Appendix B and Sec. 4.4) as
hand-written HIP kernels behind the C ABI of include/tmq.h; ``tmq`` is the
ctypes binding.  Using the package requires the built libtmq.so
(``python -m paper_0905_3331_amd.build``); there is no CPU fallback.  The
binding is loaded on first attribute access, so that the build module can be
imported without a library.
"""
_EXPORTS = ("BF16", "FP16", "FP32", "FP64", "Lattice", "SolveInfo", "TmqError", "footprint_bytes", "params",
            "solver_opts", "version")


def __getattr__(name):
    if name in _EXPORTS or name == "tmq":
        import importlib

        tmq = importlib.import_module(__name__ + ".tmq")
        return tmq if name == "tmq" else getattr(tmq, name)
    raise AttributeError(name)


__all__ = list(_EXPORTS)
