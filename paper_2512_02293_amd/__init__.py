"""MI355X (gfx950) visual-inertial bundle-adjustment step.

``binding`` holds the ctypes binding of the HIP library (include/vi_ba.h),
``synth`` the seeded synthetic workload generator, ``_build`` the hipcc build.
Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = ["binding", "synth"]
