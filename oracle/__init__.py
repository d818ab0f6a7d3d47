"""FP64 CPU oracle of the channel-emulation path -- test infrastructure only.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The library never does.
"""
