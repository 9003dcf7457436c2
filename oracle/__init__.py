"""CPU oracle of the ELAS hot path. TEST INFRASTRUCTURE ONLY.

The C sources here are the parity reference for the HIP library; they share
no code with it. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may load them.
"""
