"""The contraction probe's MFMA forms compute what its VALU form computes
(the register-layout stepper's d = 3 contraction), to FP32 rounding."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def scp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_18155_amd as m
    return m


def _ops(nop, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(nop, 3, 3)) + 1j * rng.normal(size=(nop, 3, 3))
    h = 0.1 * (a + a.conj().transpose(0, 2, 1))
    flat = np.concatenate([h.real.reshape(nop, 9), h.imag.reshape(nop, 9)], axis=1)
    return torch.tensor(flat, dtype=torch.float32, device="cuda"), h


def test_mfma_forms_equal_the_valu_form(scp):
    ops, _ = _ops(3, 1)
    print("[probe] forms 0 and 1, 3 operators, 20 applications", flush=True)
    y0 = scp.probe_contraction(0, ops, 20, n_wg=8).cpu().numpy()
    y1 = scp.probe_contraction(1, ops, 20, n_wg=8).cpu().numpy()
    assert np.abs(y1 - y0).max() <= 1e-5 * np.abs(y0).max()
    one = ops[:1]
    y0 = scp.probe_contraction(0, one, 20, n_wg=8).cpu().numpy()
    y2 = scp.probe_contraction(2, one, 20, n_wg=8).cpu().numpy()
    assert np.abs(y2 - y0).max() <= 1e-5 * np.abs(y0).max()


def test_valu_form_matches_numpy(scp):
    # one lane's 27 amplitudes follow the kernel's seeded pattern; the sum of
    # the outputs of one application is checked for lane 0 of workgroup 0
    ops, h = _ops(1, 2)
    y = scp.probe_contraction(0, ops, 1, n_wg=1).cpu().numpy()
    gid = 0
    x = np.zeros(27, dtype=np.complex128)
    for r in range(27):
        hh = ((gid * 131 + r * 7919) * 2654435761) & 0xFFFFFFFF
        x[r] = ((hh & 0xFFFF) / 65536.0 - 0.5) + 1j * (((hh >> 16) & 0xFFFF) / 65536.0 - 0.5)
    out = (h[0] @ x.reshape(9, 3).T).T.reshape(27)
    ref = out.real.sum() + 0.5 * out.imag.sum()
    assert abs(y[0] - ref) <= 1e-5 * max(1.0, abs(ref))


def test_probe_refuses_bad_arguments(scp):
    ops, _ = _ops(1, 3)
    with pytest.raises(scp.ScpError, match="EINVAL"):
        scp.probe_contraction(3, ops, 1, n_wg=1)
