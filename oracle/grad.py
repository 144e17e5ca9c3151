"""Oracle gradient of the pseudo-energy by reverse-mode automatic differentiation.

TEST INFRASTRUCTURE ONLY.  E (reading R8 of ``fftroute``) is a real polynomial
in the orbital coefficients c, c* and a smooth function of the Jastrow
parameters; torch.autograd differentiates the oracle's own discrete energy, so
the result is the exact gradient of that discrete functional.  It is pinned to
central finite differences in tests/test_oracle_grad.py.

Convention: grad_c = dE/dRe(c) + i dE/dIm(c) = 2 dE/dc* (Wirtinger), for the
coefficients shared by both spin channels (TC mode, chi = phi = c); dA and dC
are the partial derivatives with A_par, A_anti, C_par, C_anti independent.

Biorthogonal mode (energy_and_grad_bitc): the gradients with respect to the right and the left
coefficients of the energy Re sum f <chi| T + h2/2 + h3/3 |phi> (reading R8), with the pair taken
as given (biorthonormalised once beforehand, not differentiated through).

Spin-polarised input (energy_and_grad_polarized, TC mode): one orbital set per spin channel, so one
gradient 2 dE/dc* per channel.  With two equal channels they add up to the unpolarised gradient, whose
coefficients both channels share.  energy_and_grad_bitc_polarized: the biorthogonal mode with one
right/left pair per channel, each taken as given.
"""
from __future__ import annotations

import torch

from .fftroute import Problem, ALL_TERMS, RD, CD, biorthogonalize_coeffs


def energy_and_grad(w, terms=ALL_TERMS, div_correction=True, with_kinetic=True, reading="printed"):
    coeff = [torch.as_tensor(c, dtype=CD).clone().requires_grad_(True) for c in w.right]
    A = torch.as_tensor(w.A, dtype=RD).clone().requires_grad_(True)
    C = torch.as_tensor(w.C, dtype=RD).clone().requires_grad_(True)
    pr = Problem(w, A=A, C=C, coeff=coeff, div_correction=div_correction, reading=reading)
    E = pr.energy(terms=terms, with_kinetic=with_kinetic)
    gc = torch.autograd.grad(E, coeff + [A, C])
    return float(E.detach()), [g.detach().numpy() for g in gc[:-2]], gc[-2].numpy(), gc[-1].numpy()


def energy(w, coeff=None, A=None, C=None, terms=ALL_TERMS, div_correction=True, with_kinetic=True,
           reading="printed"):
    with torch.no_grad():
        pr = Problem(w, A=A, C=C, coeff=None if coeff is None else [torch.as_tensor(c, dtype=CD) for c in coeff],
                     div_correction=div_correction, reading=reading)
        return float(pr.energy(terms=terms, with_kinetic=with_kinetic))


def bitc_pair(w):
    """The workload's right/left pair after the biorthonormalisation of Sec. 2.3 (numpy arrays)."""
    cr, cl = biorthogonalize_coeffs([torch.as_tensor(c, dtype=CD) for c in w.right],
                                    [torch.as_tensor(c, dtype=CD) for c in w.left])
    return [c.numpy() for c in cr], [c.numpy() for c in cl]


def energy_and_grad_bitc(w, right, left, terms=ALL_TERMS, div_correction=True, reading="printed"):
    """(E, grad_right, grad_left, dA, dC) of the biorthogonal-mode energy at the given pair."""
    r = [torch.as_tensor(c, dtype=CD).clone().requires_grad_(True) for c in right]
    l = [torch.as_tensor(c, dtype=CD).clone().requires_grad_(True) for c in left]
    A = torch.as_tensor(w.A, dtype=RD).clone().requires_grad_(True)
    C = torch.as_tensor(w.C, dtype=RD).clone().requires_grad_(True)
    pr = Problem(w, A=A, C=C, coeff=r, left=l, div_correction=div_correction, biorthogonalize=False,
                 reading=reading)
    E = pr.energy(terms=terms)
    g = torch.autograd.grad(E, r + l + [A, C])
    nk = len(r)
    return (float(E.detach()), [x.numpy() for x in g[:nk]], [x.numpy() for x in g[nk:2 * nk]],
            g[-2].numpy(), g[-1].numpy())


def energy_bitc(w, right, left, terms=ALL_TERMS, div_correction=True, reading="printed"):
    with torch.no_grad():
        pr = Problem(w, coeff=[torch.as_tensor(c, dtype=CD) for c in right],
                     left=[torch.as_tensor(c, dtype=CD) for c in left], div_correction=div_correction,
                     biorthogonalize=False, reading=reading)
        return float(pr.energy(terms=terms))


def energy_and_grad_polarized(w, terms=ALL_TERMS, div_correction=True, reading="printed"):
    """(E, grad_up, grad_dn, dA, dC) of a spin-polarised workload (TC mode)."""
    up = [torch.as_tensor(c, dtype=CD).clone().requires_grad_(True) for c in w.right]
    dn = [torch.as_tensor(c, dtype=CD).clone().requires_grad_(True) for c in w.right_dn]
    A = torch.as_tensor(w.A, dtype=RD).clone().requires_grad_(True)
    C = torch.as_tensor(w.C, dtype=RD).clone().requires_grad_(True)
    pr = Problem(w, A=A, C=C, coeff=up, coeff_dn=dn, div_correction=div_correction, reading=reading)
    E = pr.energy(terms=terms)
    g = torch.autograd.grad(E, up + dn + [A, C])
    nk = len(up)
    return (float(E.detach()), [x.numpy() for x in g[:nk]], [x.numpy() for x in g[nk:2 * nk]],
            g[-2].numpy(), g[-1].numpy())


def energy_polarized(w, up=None, dn=None, A=None, C=None, terms=ALL_TERMS, div_correction=True):
    with torch.no_grad():
        pr = Problem(w, A=A, C=C, coeff=None if up is None else [torch.as_tensor(c, dtype=CD) for c in up],
                     coeff_dn=None if dn is None else [torch.as_tensor(c, dtype=CD) for c in dn],
                     div_correction=div_correction)
        return float(pr.energy(terms=terms))


def bitc_pair_polarized(w):
    """Both channels' right/left pairs after the biorthonormalisation of Sec. 2.3 (numpy arrays):
    (right_up, left_up, right_dn, left_dn)."""
    ru, lu = bitc_pair(w)
    rd, ld = biorthogonalize_coeffs([torch.as_tensor(c, dtype=CD) for c in w.right_dn],
                                    [torch.as_tensor(c, dtype=CD) for c in w.left_dn])
    return ru, lu, [c.numpy() for c in rd], [c.numpy() for c in ld]


def energy_and_grad_bitc_polarized(w, ru, lu, rd, ld, terms=ALL_TERMS, div_correction=True, reading="printed"):
    """(E, grad_right_up, grad_left_up, grad_right_dn, grad_left_dn, dA, dC) of the spin-polarised
    biorthogonal-mode energy at the given pairs."""
    sets = [[torch.as_tensor(c, dtype=CD).clone().requires_grad_(True) for c in x] for x in (ru, lu, rd, ld)]
    A = torch.as_tensor(w.A, dtype=RD).clone().requires_grad_(True)
    C = torch.as_tensor(w.C, dtype=RD).clone().requires_grad_(True)
    pr = Problem(w, A=A, C=C, coeff=sets[0], left=sets[1], coeff_dn=sets[2], left_dn=sets[3],
                 div_correction=div_correction, biorthogonalize=False, reading=reading)
    E = pr.energy(terms=terms)
    flat = [x for st in sets for x in st]
    g = torch.autograd.grad(E, flat + [A, C])
    nk = len(ru)
    out = [[x.numpy() for x in g[i * nk:(i + 1) * nk]] for i in range(4)]
    return (float(E.detach()), *out, g[-2].numpy(), g[-1].numpy())
