"""MI355X-native local-energy engine for autoregressive neural-quantum-state VMC.

The compute path lives in the HIP library ``libelocal.so`` (C ABI in
``include/elocal.h``); ``paper_2506_07430_amd.elocal`` is its Python binding and
``paper_2506_07430_amd.synth`` draws seeded synthetic inputs.
"""
