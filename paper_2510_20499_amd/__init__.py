"""Bound propagation and double probing over sparse MILP matrices on MI355X.

The compute path is the HIP library ``libbp.so`` built from ``csrc/``; the
Python module :mod:`paper_2510_20499_amd.bp` only marshals arguments to its
C entry points.
"""
