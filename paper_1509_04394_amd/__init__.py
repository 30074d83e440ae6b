"""fz: fused video-kernel chains on MI355X (gfx950).

``paper_1509_04394_amd.fz`` is the binding of the C ABI in include/fz.h;
``paper_1509_04394_amd.synth`` makes seeded synthetic video.  Importing the
package loads nothing; the library is loaded on first use of the binding.
"""
__all__ = ["fz", "synth"]
