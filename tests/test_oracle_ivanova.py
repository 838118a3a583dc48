"""Pins of the oracle's Ivanova effective surfaces (Part II eq:IvanovaAij with
the analytic partition-of-unity gradients of the appendix "Full Expressions
For Partitions of Unity And Their Gradients").

- grad psi_j(x_i) against central differences of psi_j(x) = W(x - x_j, H_i) /
  sum_k W(x - x_k, H_i), evaluated by brute force over all particles (H held
  at H_i, as the appendix does);
- the gradients of the partition of unity sum to zero at every particle;
- A_ij = -A_ji bitwise;
- on a perfect lattice the normalisation gradients vanish and the surfaces
  close (sum_j A_ij = 0), as the thesis shows for regular configurations;
- on an irregular set the thesis' identity sum_j A_ij = -sum_j V_j grad
  psi_i(x_j) holds;
- one transport step with these surfaces conserves photons and differs from
  the Hopkins step.
"""
import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module")
def irregular(orc):
    x = workloads.jittered_lattice(8, 0.25, 301)
    geo = oracle.build_geometry(x)
    return geo, oracle.ivanova_sums(geo)


def kernel_W(r, H):
    q = r / H
    a = np.maximum(1.0 - q, 0.0)
    b = np.maximum(0.5 - q, 0.0)
    return (16.0 / np.pi) / H ** 3 * (a ** 3 - 4.0 * b ** 3)


def psi_bruteforce(geo, j, x, Hi):
    d = geo.x - x
    d -= np.round(d)                                     # periodic unit box
    W = kernel_W(np.sqrt((d * d).sum(-1)), Hi)
    return W[j] / W.sum()


def test_grad_psi_against_central_differences(irregular):
    geo, gsum = irregular
    g = workloads.rng(302)
    worst = 0.0
    for i in g.choice(geo.n, 12, replace=False):
        Hi = geo.H[i]
        nbrs = geo.gidx[geo.gptr[i]:geo.gptr[i + 1]]
        d = geo.x[nbrs] - geo.x[i]
        d -= np.round(d)
        # away from the edge of the support, where (1 - q)^3 has a large third
        # derivative relative to its first and the differences lose accuracy
        nbrs = nbrs[np.sqrt((d * d).sum(-1)) < 0.9 * Hi]
        for j in g.choice(nbrs, 4, replace=False):
            an = oracle.grad_psi(geo, gsum, i, j)
            fd = np.zeros(3)
            dlt = 1e-6 * Hi
            for a in range(3):
                e = np.zeros(3)
                e[a] = dlt
                fd[a] = (psi_bruteforce(geo, j, geo.x[i] + e, Hi)
                         - psi_bruteforce(geo, j, geo.x[i] - e, Hi)) / (2 * dlt)
            worst = max(worst, np.abs(an - fd).max() / np.abs(fd).max())
    assert worst < 1e-7


def test_gradients_of_the_partition_of_unity_sum_to_zero(irregular):
    geo, gsum = irregular
    for i in range(0, geo.n, 37):
        terms = [oracle.grad_psi(geo, gsum, i, i)]
        terms += [oracle.grad_psi(geo, gsum, i, j) for j in geo.gidx[geo.gptr[i]:geo.gptr[i + 1]]]
        terms = np.array(terms)
        assert np.abs(terms.sum(0)).max() < 1e-12 * np.abs(terms).max()


def test_antisymmetry_bitwise(irregular):
    geo, gsum = irregular
    for k in range(0, geo.n, 29):
        for l in geo.sidx[geo.sptr[k]:geo.sptr[k + 1]]:
            assert np.array_equal(oracle.surface_ivanova(geo, gsum, k, l),
                                  -oracle.surface_ivanova(geo, gsum, l, k))


def test_perfect_lattice_closes(orc):
    n = 8
    ax = (np.arange(n) + 0.5) / n
    x = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    geo = oracle.build_geometry(x)
    gsum = oracle.ivanova_sums(geo)
    scale = np.abs(oracle.surface_ivanova(geo, gsum, 0, geo.sidx[geo.sptr[0]])).max()
    assert np.abs(gsum).max() < 1e-10 * np.abs(gsum).max(initial=1.0)
    for k in range(0, geo.n, 41):
        tot = sum(oracle.surface_ivanova(geo, gsum, k, l) for l in geo.sidx[geo.sptr[k]:geo.sptr[k + 1]])
        assert np.abs(tot).max() < 1e-12 * scale


def test_closure_identity_on_irregular_sets(irregular):
    # sum_{j != i} A_ij = -sum_j V_j grad psi_i(x_j), the sum on the right over
    # every particle whose kernel reaches x_i, i itself included
    geo, gsum = irregular
    for i in range(0, geo.n, 31):
        nb = geo.sidx[geo.sptr[i]:geo.sptr[i + 1]]
        A = np.array([oracle.surface_ivanova(geo, gsum, i, j) for j in nb])
        lhs = A.sum(0)
        rhs = -geo.V[i] * oracle.grad_psi(geo, gsum, i, i)
        for j in nb:
            rhs = rhs - geo.V[j] * oracle.grad_psi(geo, gsum, j, i)
        scale = np.abs(A).max()
        assert np.abs(lhs - rhs).max() < 1e-12 * scale
        assert np.abs(lhs).max() > 1e-6 * scale           # not closed on irregular sets


def test_step_conserves_and_differs_from_hopkins(orc):
    x = workloads.jittered_lattice(10, 0.1, 303)
    g = workloads.rng(304)
    E = 1.0 + 0.3 * np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
    U0 = np.zeros((x.shape[0], 1, 4))
    U0[:, 0, 0] = E
    U0[:, 0, 1:] = 0.05 * E[:, None] * g.normal(size=(x.shape[0], 3))
    geo = oracle.build_geometry(x)
    out, info = oracle.step(geo, None, U0, ivanova=True)
    assert not info["counts"].any()
    Q0, Q1 = oracle.photon_total(geo, U0), oracle.photon_total(geo, out)
    assert np.abs(Q1 / Q0 - 1).max() < 1e-13
    hop, _ = oracle.step(geo, None, U0)
    assert np.abs(out - hop).max() > 1e-6 * np.abs(hop).max()
