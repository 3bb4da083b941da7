"""Orbital subsets for sampled checks at full size (test helper: index bookkeeping only).

Every term of the residuals and of the energy sums a core or virtual index only
through a contraction that ends on an amplitude: the Hamiltonian is normal ordered,
and the density and cumulant factors carry active indices alone.  Amplitudes that
vanish outside a chosen set of core and virtual orbitals therefore make every
residual element whose indices lie in (chosen cores + all actives + chosen virtuals)
equal to the same element of the problem restricted to those orbitals.  The same
holds for the correlation energy.  tests/test_subset_cpu.py checks this with the
oracle on both sides; the full-size GPU test relies on it.
"""
import numpy as np


def orbitals(nc, na, cores, virts):
    """Full orbital numbers of the subset, in core, active, virtual order."""
    return np.concatenate([np.asarray(cores, dtype=np.int64), nc + np.arange(na),
                           nc + na + np.asarray(virts, dtype=np.int64)])


def restrict(f, B, nc, na, cores, virts):
    """f and B restricted to the subset's orbitals."""
    orb = orbitals(nc, na, cores, virts)
    return f[np.ix_(orb, orb)], np.ascontiguousarray(B[:, orb][:, :, orb])


def hole_map(nc, na, cores):
    """Full hole positions (core + active) of the subset's hole positions."""
    return np.concatenate([np.asarray(cores, dtype=np.int64), nc + np.arange(na)])


def particle_map(na, virts):
    """Full particle positions (active + virtual) of the subset's particle positions."""
    return np.concatenate([np.arange(na), na + np.asarray(virts, dtype=np.int64)])


def embed(T1s, T2s, hm, pm, nH, nP):
    """Full-size amplitudes that equal the subset's on its positions and vanish elsewhere."""
    T1 = np.zeros((nH, nP))
    T2 = np.zeros((nH, nH, nP, nP))
    T1[np.ix_(hm, pm)] = T1s
    T2[np.ix_(hm, hm, pm, pm)] = T2s
    return T1, T2
