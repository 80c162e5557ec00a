"""MI355X-native resonant discrete diffusion Monte Carlo (rDDMC) Lyman-alpha transfer.

* ``media``  -- seeded synthetic media and sources (no transport arithmetic)
* ``rddmc``  -- Python binding of the C ABI in include/rddmc.h (librddmc.so, HIP, gfx950)
* ``build``  -- compiles librddmc.so in-tree with hipcc
"""
__all__ = ["media", "rddmc", "build"]
