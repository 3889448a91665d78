"""Plain FP64 CPU oracle of the Penning-trap FMM hot path.

Test infrastructure only: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.
"""
