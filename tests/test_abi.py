"""The C-ABI library loads, exports every symbol the header declares, and its host-only routines
(FP64 eigensolvers used for the FNS and Davidson subspace steps) work without a GPU."""
import pathlib
import re

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parents[1]


def _declared():
    src = (ROOT / "include" / "fnscc.h").read_text()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_declared_symbols():
    from paper_2506_06805_amd import fnscc
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(fnscc.lib, name), name
        assert name in fnscc.EXPORTED, name


def test_host_hermitian_eig_matches_definition():
    from paper_2506_06805_amd import fnscc
    rng = np.random.default_rng(0)
    for n in (1, 2, 3, 17, 64):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        H = A + A.conj().T
        w, V = fnscc.host_zheev(H)
        assert np.all(np.diff(w) >= 0)
        assert np.abs(H @ V - V * w).max() < 1e-12 * max(1, np.abs(H).max()) * n
        assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12 * n
    # degenerate spectrum and a diagonal matrix
    w, V = fnscc.host_zheev(np.diag([2.0, 1.0, 2.0, 0.5]).astype(complex))
    assert np.allclose(w, [0.5, 1.0, 2.0, 2.0])


def test_host_general_eig_matches_definition():
    from paper_2506_06805_amd import fnscc
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 33, 120):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        w, V = fnscc.host_zgeev(A)
        assert np.abs(A @ V - V * w).max() < 1e-11 * n
        assert np.abs(np.linalg.norm(V, axis=0) - 1).max() < 1e-12
    # upper triangular input: eigenvalues are the diagonal
    T = np.triu(rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6)))
    w, _ = fnscc.host_zgeev(T)
    assert np.abs(np.sort_complex(w) - np.sort_complex(np.diag(T))).max() < 1e-12


def test_bad_arguments_are_rejected_without_gpu():
    from paper_2506_06805_amd import fnscc
    assert fnscc.lib.fc_host_zheev(-1, None, None) == fnscc.FC_EARG
    assert fnscc.lib.cd_integrals(None, 1, 1, 1, None, None, 0, 0, 0, None) == fnscc.FC_EARG
    assert fnscc.lib.ccsd_solve(None, 1, None, None, None, None, None) == fnscc.FC_EARG
