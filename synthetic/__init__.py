"""Seeded synthetic inputs shared by the oracle and the GPU path.

Holds lattices, force constants and workload definitions only; none of the
phonon / linewidth / conductivity arithmetic lives here.
"""
