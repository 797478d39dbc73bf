"""MI355X-native fast Fourier spectral method for the linearized Boltzmann
collision operator L[h] = Q(M,h) + Q(h,M) (VHS gases), after Yin, Cai and
Wang, arXiv 2503.09580.

The compute path is the HIP library ``liblincoll.so`` (C ABI, declared in
``include/lincoll.h``); ``paper_2503_09580_amd.lincoll`` is its thin Python
binding.  Importing this package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
