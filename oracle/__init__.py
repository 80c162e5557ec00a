"""CPU oracle for rDDMC Lyman-alpha transfer -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 implementations of what the GPU library computes, written
from the paper (Smith, Tsang, Bromm & Milosavljevic 2017, "Discrete diffusion
Lyman alpha radiative transfer").  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import anything in this package; the
product library never does, and shares no code with it (the only shared
module is the input generator ``paper_1709_10187_amd.media``, which holds no
transport arithmetic).

Modules
-------
linemath   Voigt profile (eq. 12), its integral (eq. 13), bin-averaged opacity (eq. 14)
tables     FP64 leakage coefficients (eqs. 10, 11, the vacuum/thin-face rate of the
           hybrid section), Doppler-shifted neighbour opacities (Sec. 2.5)
chain      O2: exact expected escape spectrum / steps / time moments of the
           pure-DDMC continuous-time Markov chain (sparse linear solves)
walk       O1: literal Monte Carlo walker (min over exponential distances,
           eqs. 15-16) in plain C, FP64, xoshiro256** streams
analytic   closed forms: Neufeld slab spectrum (eq. 33), the sphere spectrum derived
           from eqs. 25 and 28, grey-chain first-passage results
philox     Philox4x32-10 written from its published definition (for paired tests)
"""
