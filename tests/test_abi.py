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


def test_binding_refuses_bad_tensors_before_any_call():
    """The binding checks dtype, shape and device before a pointer reaches the library (a host
    tensor, a short tensor or the wrong element type would be read past its end by a kernel)."""
    import types

    import pytest
    import torch

    from paper_2506_06805_amd import fnscc
    o, v = 3, 5
    ints = types.SimpleNamespace(o=o, v=v, dim=o + o * (o - 1) // 2 * v)
    eps = np.linspace(-1, 1, o + v)
    with pytest.raises(ValueError, match="L must be"):
        fnscc.cd_integrals(None, eps, np.zeros((2, o + v, o + v - 1), np.complex128), o)
    with pytest.raises(ValueError, match="neither complex128 nor complex64"):
        fnscc.cd_integrals(None, eps, np.zeros((2, o + v, o + v)), o)
    with pytest.raises(ValueError, match="GPU tensor"):
        fnscc.cd_integrals(None, eps, torch.zeros((2, o + v, o + v), dtype=torch.complex128), o)
    t1 = torch.zeros((o, v), dtype=torch.complex128)
    t2 = torch.zeros((o, o, v, v), dtype=torch.complex128)
    with pytest.raises(ValueError, match="GPU tensor"):
        fnscc.ccsd_residual(None, ints, t1, t2)
    with pytest.raises(ValueError, match="GPU tensor"):
        fnscc.amps_create(None, ints, t1, t2)
    with pytest.raises(ValueError, match="GPU tensor"):
        fnscc.ladder(None, ints, t2)
    with pytest.raises(ValueError):
        fnscc.ipeom_sigma(None, ints, None, torch.zeros((2, ints.dim), dtype=torch.complex128))
    with pytest.raises(ValueError):
        fnscc.ipeom_sigma_left(None, ints, None, np.zeros((2, ints.dim), np.complex128))
    with pytest.raises(ValueError):
        fnscc.zgemm(None, "N", "N", torch.zeros((2, 2), dtype=torch.float64), torch.zeros((2, 2)))
    with pytest.raises(ValueError):
        fnscc.ccsd_opts(t1_init=t1)


def test_binding_checks_shapes_and_dtypes_of_device_tensors(monkeypatch):
    """Shape and dtype checks act on tensors that claim to be on the GPU (device check passed)."""
    import types

    import pytest
    import torch

    from paper_2506_06805_amd import fnscc
    o, v = 3, 5
    ints = types.SimpleNamespace(o=o, v=v, dim=o + o * (o - 1) // 2 * v)

    real_require = fnscc._require

    def require(t, name, dtypes, shape=None):
        # a CPU tensor standing in for a device one: check everything but the device
        if isinstance(t, torch.Tensor) and t.device.type == "cpu":
            if t.dtype not in dtypes:
                raise ValueError(f"{name}: dtype {t.dtype} not accepted")
            if shape is not None and tuple(t.shape) != tuple(shape):
                raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")
            return t
        return real_require(t, name, dtypes, shape)

    monkeypatch.setattr(fnscc, "_require", require)
    with pytest.raises(ValueError, match="shape"):
        fnscc.ipeom_sigma(None, ints, None, torch.zeros((2, ints.dim - 1), dtype=torch.complex128))
    with pytest.raises(ValueError, match="dtype"):
        fnscc.ipeom_sigma(None, ints, None, torch.zeros((2, ints.dim), dtype=torch.complex64))
    with pytest.raises(ValueError, match="shape"):
        fnscc.ccsd_residual(None, ints, torch.zeros((o, v), dtype=torch.complex128),
                            torch.zeros((o, o, v, v - 1), dtype=torch.complex128))
    with pytest.raises(ValueError, match="dtype"):
        fnscc.ladder(None, ints, torch.zeros((o, o, v, v), dtype=torch.complex64))
