"""MI355X-native Kob-Andersen binary Lennard-Jones MD hot path (arXiv:2001.07089).

The work runs in the HIP library ``_lib/libkamd.so`` behind the C ABI declared
in ``include/kamd.h``; ``paper_2001_07089_amd.md`` is the thin ctypes binding
with the same function names.  PyTorch is used only for device memory and
streams.
"""
__all__ = ["md", "workload"]
