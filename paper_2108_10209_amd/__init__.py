"""Noise2Fast per-image train-and-denoise loop for MI355X (gfx950).

The compute path is the HIP library `libn2f.so` behind the C ABI declared in
include/n2f.h; `paper_2108_10209_amd.n2f` is its thin ctypes binding and
`paper_2108_10209_amd.synth` makes seeded synthetic inputs.  Importing this
package loads nothing.
"""
