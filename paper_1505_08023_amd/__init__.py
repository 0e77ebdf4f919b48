"""MI355X (gfx950) library for the MiniFE-style finite-element hot path.

The HIP library libmfe.so (C ABI in include/mfe.h) does the work; this
package only binds it.  `mfe` (Context, Problem) needs PyTorch for device
memory and streams; `_lib` is the raw ctypes binding.
"""
