"""The device natural logarithm and reciprocal of the direct-interaction, P2L and M2QBXL kernels
(gq_device_math) against numpy over their input range.

The logarithm is table-driven (128 entries, a degree-7 log1p series, a two-part log 2): its
absolute error stays near one ulp of 1 for arguments near 1 and one ulp of |log x| elsewhere.
The reciprocal refines the hardware estimate by two Newton steps: within an ulp of 1/x.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib_ctx():
    from paper_1801_04070_amd import QBXFMM
    return QBXFMM(device=0)


def _sweep(rng):
    # every binade of the normal doubles, mantissas at the table's bin edges, bin centers and
    # random points, plus values next to 1 (where log x is small and the series does the work)
    e = np.arange(-1021, 1023)
    j = np.arange(129)
    edges = 1.0 + j / 128.0
    mids = 1.0 + (j[:-1] + 0.5) / 128.0
    rand = rng.uniform(1.0, 2.0, 400)
    mant = np.concatenate([edges[:-1], np.nextafter(edges[1:], 0), mids, rand])
    x = np.ldexp(mant[None, :], e[:, None]).ravel()
    near1 = 1.0 + np.concatenate([np.arange(-4000, 4001) * 2.0 ** -52,
                                  rng.uniform(-2 ** -7, 2 ** -7, 20000)])
    return np.concatenate([x, near1])


def test_device_log_accuracy():
    from paper_1801_04070_amd import _lib
    q = _lib_ctx()
    x = _sweep(np.random.default_rng(1))
    got = q.device_math(_lib.GQ_MATH_LOG, torch.as_tensor(x, device="cuda:0")).cpu().numpy()
    ref = np.log(x)
    err = np.abs(got - ref)
    ulp_ref = np.spacing(np.maximum(np.abs(ref), 1.0))
    print(f"log: max error {(err / ulp_ref).max():.2f} ulp of max(|log x|, 1)")
    assert (err <= 2.0 * ulp_ref).all()
    # exact at powers of two' logs up to the split of log 2 (k log 2 for integer k)
    k = np.arange(-1000, 1001)
    got2 = q.device_math(_lib.GQ_MATH_LOG,
                         torch.as_tensor(np.ldexp(1.0, k), device="cuda:0")).cpu().numpy()
    assert (np.abs(got2 - k * np.log(2.0)) <= 2.0 * np.spacing(np.maximum(np.abs(k) * 0.7, 1))).all()


def test_device_reciprocal_accuracy():
    from paper_1801_04070_amd import _lib
    q = _lib_ctx()
    rng = np.random.default_rng(2)
    x = _sweep(rng)
    x = x[np.abs(x) < 2.0 ** 1021]  # 1/x stays a normal double
    x = np.concatenate([x, -x])
    got = q.device_math(_lib.GQ_MATH_RCP, torch.as_tensor(x, device="cuda:0")).cpu().numpy()
    ref = 1.0 / x
    ulps = np.abs(got - ref) / np.spacing(np.abs(ref))
    print(f"rcp: max error {ulps.max():.2f} ulp")
    assert ulps.max() <= 1.0
