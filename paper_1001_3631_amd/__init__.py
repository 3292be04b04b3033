"""MI355X engine for the m-mode Teukolsky Lax-Wendroff evolution.

The HIP library (libteuk.so, C ABI in include/teuk.h) is loaded lazily by
paper_1001_3631_amd.engine / _lib; importing the package itself loads nothing.
"""

__all__ = ["engine", "workloads"]
