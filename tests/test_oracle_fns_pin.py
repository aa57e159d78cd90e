"""Pin of the oracle's frozen-natural-spinor steps at a threshold that really truncates (Eq. 24-28).

Everything on the reference side is formed by brute force in the Fock space of a tiny spinor
system, from the operator definitions alone:

* the first-order (MP2) wavefunction |Psi1> = sum_K |K> <K|H|Phi0> / (E0 - E_K) over the doubly
  excited determinants K, with E_K - E0 = eps_a + eps_b - eps_i - eps_j (the diagonal Fock
  operator of the reference as the zeroth-order Hamiltonian);
* its virtual one-body density rho_ab = <Psi1|a+_b a_a|Psi1>, the matrix <a|rho|b> of the
  one-particle density operator, whose eigenvectors are the natural spinors;
* the rotated spinors a~+_k = sum_a U_ak a+_a, with the density <Psi1|a~+_l a~_k|Psi1> and the
  one-body Cholesky operators <0|a~_k L^P a~+_l|0> taken between them.

The oracle's D_vv, its kept subspace and its transformed Cholesky vectors must agree with these.
Two plausible slips, a transposed (= conjugated) density and a conjugated rotation, are planted in
copies of the oracle functions below and must each fail the pin.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fns
from oracle import fockspace as fsm
from paper_2506_06805_amd import synth

O, V, NCD = 3, 9, 14


@pytest.fixture(scope="module")
def system():
    inst = synth.make_instance(O, V, NCD, seed=21, kappa=0.8, fns_gamma=4.0)
    fs = fsm.FockSpace(O + V)
    H = fsm.build_h(fs, inst.eps, inst.L, O)
    psi1 = first_order_wavefunction(fs, H, inst.eps, O)
    rho = np.array([[np.vdot(psi1, fs.ad(O + b) @ (fs.a(O + a) @ psi1)) for b in range(V)] for a in range(V)])
    return inst, fs, psi1, rho


def first_order_wavefunction(fs, H, eps, o):
    """|Psi1> = sum over doubly excited determinants of <K|H|Phi0> / (eps_i + eps_j - eps_a - eps_b)."""
    n = fs.n
    phi0 = fsm.reference(fs, o)
    hphi = H @ phi0
    out = np.zeros_like(hphi)
    occ_mask = (1 << o) - 1
    for s in range(fs.dim):
        if bin(s).count("1") != o:
            continue
        holes = [i for i in range(o) if not (s >> i) & 1]
        parts = [p for p in range(o, n) if (s >> p) & 1]
        if len(holes) == 2 and len(parts) == 2:
            d = eps[holes[0]] + eps[holes[1]] - eps[parts[0]] - eps[parts[1]]
            out[s] = hphi[s] / d
        elif s != occ_mask:
            # singles vanish with a diagonal Fock operator (Brillouin); higher excitations are not
            # reached by a two-body H from the reference
            assert abs(hphi[s]) < 1e-12
    return out


def rotated_annihilators(fs, U, o):
    """a~_k = sum_a conj(U_ak) a_a for the columns k of U (virtual spinors a = o + row)."""
    return [sum(np.conj(U[a, k]) * fs.a(o + a) for a in range(U.shape[0])) for k in range(U.shape[1])]


def one_body(fs, Lp):
    n = fs.n
    return sum(Lp[p, q] * (fs.ad(p) @ fs.a(q)) for p in range(n) for q in range(n) if Lp[p, q] != 0)


def pin_violations(inst, fs, psi1, rho, thresh, vv_density=fns.vv_density, truncate=fns.truncate):
    """Largest deviations of the oracle's FNS quantities from their Fock-space definitions."""
    o, v = inst.o, inst.v
    out = {}
    D = vv_density(inst.L, inst.eps, o)
    out["density"] = np.abs(D - rho).max()
    L2, eps2, vk, n_occ, U = truncate(inst.L, inst.eps, o, thresh)
    # occupations: the eigenvalues of the Fock-space density, descending; kept = above threshold
    ref_occ = np.sort(np.linalg.eigvalsh(rho))[::-1]
    out["occupations"] = np.abs(n_occ - ref_occ).max()
    out["kept_count"] = float(vk != int(np.sum(ref_occ > thresh)))
    # the density between the rotated spinors: its spectrum is the kept occupations and the
    # kept space is invariant under rho (no leakage to the dropped natural spinors)
    ann = rotated_annihilators(fs, U, o)
    N = np.array([[np.vdot(psi1, ann[l].getH() @ (ann[k] @ psi1)) for l in range(vk)] for k in range(vk)])
    out["kept_spectrum"] = np.abs(np.sort(np.linalg.eigvalsh(N))[::-1] - ref_occ[:vk]).max()
    out["kept_trace"] = abs(np.trace(N) - ref_occ[:vk].sum())
    out["invariance"] = np.abs(rho @ U - U @ (U.conj().T @ rho @ U)).max()
    # semicanonical: the Fock operator between rotated spinors is diagonal with eps2 (Eq. 26-27)
    vac = np.zeros(fs.dim, dtype=np.complex128)
    vac[0] = 1.0
    fock = sum(inst.eps[o + a] * (fs.ad(o + a) @ fs.a(o + a)) for a in range(v))
    Fk = np.array([[np.vdot(ann[k].getH() @ vac, fock @ (ann[l].getH() @ vac)) for l in range(vk)] for k in range(vk)])
    out["semicanonical"] = np.abs(Fk - np.diag(eps2[o:])).max()
    out["occupied_eps"] = np.abs(eps2[:o] - inst.eps[:o]).max()
    # transformed Cholesky vectors: <0|a~_k L^P a~+_l|0> and <0|a_i L^P a~+_l|0>
    worst = 0.0
    for P in (0, inst.ncd // 2, inst.ncd - 1):
        Lop = one_body(fs, inst.L[P])
        kets = [ann[l].getH() @ vac for l in range(vk)]
        bras_v = [ann[k].getH() @ vac for k in range(vk)]
        bras_o = [fs.ad(i) @ vac for i in range(o)]
        ref_vv = np.array([[np.vdot(bras_v[k], Lop @ kets[l]) for l in range(vk)] for k in range(vk)])
        ref_ov = np.array([[np.vdot(bras_o[i], Lop @ kets[l]) for l in range(vk)] for i in range(o)])
        ref_vo = np.array([[np.vdot(bras_v[k], Lop @ bras_o[i]) for i in range(o)] for k in range(vk)])
        worst = max(worst, np.abs(L2[P, o:, o:] - ref_vv).max(), np.abs(L2[P, :o, o:] - ref_ov).max(),
                    np.abs(L2[P, o:, :o] - ref_vo).max(), np.abs(L2[P, :o, :o] - inst.L[P, :o, :o]).max())
    out["cholesky"] = worst
    return out


def _threshold(rho, keep):
    occ = np.sort(np.linalg.eigvalsh(rho))[::-1]
    return float(np.sqrt(occ[keep - 1] * occ[keep]))   # between the keep-th and the next occupation


def test_density_is_complex_and_spread(system):
    # the pin is only sharp if D is not real symmetric and a threshold splits its spectrum
    _, _, _, rho = system
    assert np.abs(rho - rho.T).max() > 1e-6
    occ = np.sort(np.linalg.eigvalsh(rho))[::-1]
    assert occ[0] / occ[-1] > 100


@pytest.mark.parametrize("keep", [3, 5])
def test_fns_matches_fock_space_definitions(system, keep):
    inst, fs, psi1, rho = system
    thresh = _threshold(rho, keep)
    viol = pin_violations(inst, fs, psi1, rho, thresh)
    assert viol["kept_count"] == 0.0
    scale = np.abs(rho).max()   # density-based entries relative to the density, the rest absolute
    for k in ("density", "occupations", "kept_spectrum", "kept_trace", "invariance"):
        assert viol[k] < 1e-10 * scale, (k, viol[k], scale)
    for k in ("semicanonical", "occupied_eps", "cholesky"):
        assert viol[k] < 1e-12, (k, viol[k])


def test_pin_catches_transposed_density(system):
    inst, fs, psi1, rho = system
    thresh = _threshold(rho, 4)

    def dens_t(L, eps, o):
        return fns.vv_density(L, eps, o).T

    def truncate_t(L, eps, o, th):
        D = dens_t(L, eps, o)
        n_occ, Vv = np.linalg.eigh(D)
        order = np.argsort(-n_occ, kind="stable")
        n_occ, Vv = n_occ[order], Vv[:, order]
        Vt = Vv[:, n_occ > th]
        e_new, Z = np.linalg.eigh(Vt.conj().T @ np.diag(eps[o:]) @ Vt)
        U = Vt @ Z
        L2, eps2 = fns.transform(L, eps, o, U, e_new)
        return L2, eps2, U.shape[1], n_occ, U

    viol = pin_violations(inst, fs, psi1, rho, thresh, vv_density=dens_t, truncate=truncate_t)
    scale = np.abs(rho).max()
    assert viol["density"] > 1e-2 * scale
    assert max(viol["invariance"], viol["kept_spectrum"]) > 1e-3 * scale


def test_pin_catches_conjugated_rotation(system):
    inst, fs, psi1, rho = system
    thresh = _threshold(rho, 4)

    def truncate_c(L, eps, o, th):
        U, e_new, n_occ = fns.natural_spinors(L, eps, o, th)
        L2, eps2 = fns.transform(L, eps, o, U.conj(), e_new)   # the rotation applied conjugated
        return L2, eps2, U.shape[1], n_occ, U

    viol = pin_violations(inst, fs, psi1, rho, thresh, truncate=truncate_c)
    assert viol["cholesky"] > 1e-3


def test_sparse_operators_are_consistent(system):
    # a~_k built from a unitary U: {a~_k, a~+_l} = delta_kl on the vacuum
    _, fs, _, _ = system
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((V, V)) + 1j * rng.standard_normal((V, V)))
    ann = rotated_annihilators(fs, Q[:, :3], O)
    vac = np.zeros(fs.dim, dtype=np.complex128)
    vac[0] = 1.0
    G = np.array([[np.vdot(ann[k].getH() @ vac, ann[l].getH() @ vac) for l in range(3)] for k in range(3)])
    assert np.abs(G - np.eye(3)).max() < 1e-13
    assert isinstance(ann[0], sp.spmatrix) or sp.issparse(ann[0])
