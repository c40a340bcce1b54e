"""GenCD Propose/Update hot path for MI355X (gfx950).

The compute runs in the HIP library ``libgencd`` built from ``csrc/``; the
Python layer only marshals arguments (see ``gencd``).
"""
