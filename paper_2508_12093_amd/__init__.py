"""MI355X-native RNS-CKKS encrypted statistics (PP-STAT hot path).

Importing the package does not load the native library; ``paper_2508_12093_amd.ffi``
does, and fails loudly when ``libppstat.so`` has not been built.
"""
