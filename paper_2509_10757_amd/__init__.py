"""MI355X-native tracking correspondence search (FastTrack, arXiv 2509.10757).

The compute path is the HIP library libfasttrack.so (include/ft.h); the Python
side only marshals arguments (`binding`).  Import `binding` explicitly: this
package import stays free of torch and of the library so that CPU-only tools
can import submodules such as `build`.
"""
__all__ = ["binding", "build"]
