"""Oracle gradient of the pseudo-energy by reverse-mode automatic differentiation.

TEST INFRASTRUCTURE ONLY.  E (reading R8 of ``fftroute``) is a real polynomial
in the orbital coefficients c, c* and a smooth function of the Jastrow
parameters; torch.autograd differentiates the oracle's own discrete energy, so
the result is the exact gradient of that discrete functional.  It is pinned to
central finite differences in tests/test_oracle_grad.py.

Convention: grad_c = dE/dRe(c) + i dE/dIm(c) = 2 dE/dc* (Wirtinger), for the
coefficients shared by both spin channels (TC mode, chi = phi = c); dA and dC
are the partial derivatives with A_par, A_anti, C_par, C_anti independent.
"""
from __future__ import annotations

import torch

from .fftroute import Problem, ALL_TERMS, RD, CD


def energy_and_grad(w, terms=ALL_TERMS, div_correction=True, with_kinetic=True):
    coeff = [torch.as_tensor(c, dtype=CD).clone().requires_grad_(True) for c in w.right]
    A = torch.as_tensor(w.A, dtype=RD).clone().requires_grad_(True)
    C = torch.as_tensor(w.C, dtype=RD).clone().requires_grad_(True)
    pr = Problem(w, A=A, C=C, coeff=coeff, div_correction=div_correction)
    E = pr.energy(terms=terms, with_kinetic=with_kinetic)
    gc = torch.autograd.grad(E, coeff + [A, C])
    return float(E.detach()), [g.detach().numpy() for g in gc[:-2]], gc[-2].numpy(), gc[-1].numpy()


def energy(w, coeff=None, A=None, C=None, terms=ALL_TERMS, div_correction=True, with_kinetic=True):
    with torch.no_grad():
        pr = Problem(w, A=A, C=C, coeff=None if coeff is None else [torch.as_tensor(c, dtype=CD) for c in coeff],
                     div_correction=div_correction)
        return float(pr.energy(terms=terms, with_kinetic=with_kinetic))
