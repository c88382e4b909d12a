"""dp_force_error_noalloc (the audit reduction with its partial sums in a
fixed device array) against dp_force_error, through the C ABI: two calls in
a row on one GPU, the second with fewer atoms, each equal to the allocating
call's result (the same partial sums added in the same order; the square
root is taken on the device instead of the host, so the RMSE may differ in
its last bit) and to the definition evaluated on the host."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(rng, n):
    import torch
    a = rng.normal(0.0, 0.05, size=(n, 3))
    b = a + rng.normal(0.0, 1e-3, size=(n, 3)) * (rng.random((n, 1)) < 0.5)
    dev = torch.device("cuda:0")
    return a, b, torch.tensor(a, device=dev), torch.tensor(b, device=dev)


def test_noalloc_matches_allocating_call_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_07276_amd import binding
    rng = np.random.default_rng(11)
    out = torch.full((2,), -1.0, dtype=torch.float64, device="cuda:0")
    for n in (40000, 37):
        print(f"case: dp_force_error_noalloc vs dp_force_error, n={n}", flush=True)
        a, b, da, db = _case(rng, n)
        rmse, mx = binding.force_error(da, db)
        binding.force_error_noalloc(da, db, out)
        torch.cuda.synchronize()
        r2, m2 = out.cpu().numpy()
        d = a - b
        ref_rmse = np.sqrt((d * d).sum() / (3 * n))
        print(f"  rmse {rmse:.17g} / {r2:.17g} (host {ref_rmse:.17g}), max {mx:.17g} / {m2:.17g}",
              flush=True)
        assert m2 == mx == np.abs(d).max()
        assert abs(r2 - rmse) <= 2.0 * np.spacing(rmse)
        assert abs(r2 - ref_rmse) <= 1e-12 * ref_rmse
    binding.force_error_noalloc(da[:0], db[:0], out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), [0.0, 0.0])


def test_noalloc_rejects_bad_sizes():
    import ctypes
    from paper_2604_07276_amd import binding
    lib = binding.load_library()
    dummy = ctypes.c_void_p(16)
    assert lib.dp_force_error_noalloc(dummy, dummy, -1, dummy, None) == -1
    assert lib.dp_force_error_noalloc(dummy, dummy, 700000001, dummy, None) == -1
    assert b"DP_FORCE_ERROR_MAX_ATOMS" in lib.dp_last_error()
    assert lib.dp_force_error_noalloc(None, dummy, 5, dummy, None) == -1
    assert lib.dp_force_error_noalloc(dummy, dummy, 5, None, None) == -1
