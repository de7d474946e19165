"""The masked error's entry point that allocates nothing (its scratch is a
static device array) against stmf_masked_error on the same inputs: two calls
in a row, the second on a smaller input, every result bit-identical."""
import ctypes as C

import numpy as np
import pytest

from paper_2205_06619_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2205_06619_amd import stmf
    return stmf


def _case(m, n, r, seed):
    rng = np.random.default_rng(seed)
    U = rng.normal(0, 1, (m, r)).astype(np.float32)
    V = rng.normal(0, 1, (r, n)).astype(np.float32)
    R = (rng.normal(0, 2, (m, n)) * np.exp(rng.normal(0, 0.5, (1, n)))).astype(np.float32)
    M = synth.fix_empty_lines((rng.random((m, n)) >= 0.4).astype(np.uint8), rng)
    R[M == 0] = np.nan
    return R, M, U, V


def _dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def _call_abi(S, R, M, U, V, err, td):
    import torch
    m, n = R.shape
    r = U.shape[1]
    st = S.lib.stmf_masked_error_noalloc(C.c_void_p(R.data_ptr()), C.c_void_p(M.data_ptr()),
                                         C.c_void_p(U.data_ptr()), C.c_void_p(V.data_ptr()),
                                         m, n, r, C.c_void_p(err.data_ptr()),
                                         C.c_void_p(td.data_ptr()),
                                         C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def test_noalloc_matches_workspace_entry_point_twice(S):
    import torch
    for m, n, r, seed in [(700, 1900, 6, 1), (130, 257, 3, 2)]:
        print(f"noalloc masked error {m}x{n} r={r}", flush=True)
        R, M, U, V = _dev(*_case(m, n, r, seed))
        err = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        td = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        assert _call_abi(S, R, M, U, V, err, td) == S.STMF_OK
        e_ref, td_ref = S.stmf_masked_error(R, M, U, V)
        torch.cuda.synchronize()
        assert float(err.cpu()[0]) == float(e_ref.cpu()[0])
        np.testing.assert_array_equal(td.cpu().numpy(), td_ref.cpu().numpy())


def test_noalloc_rejects_shapes_beyond_its_scratch(S):
    import torch
    # 8192 x 8256 needs 64 x 8256 partials, above the 2^20 the scratch holds;
    # the check comes before any work, so the pointers are never read
    d = torch.zeros(4, dtype=torch.float32, device="cuda")
    p = C.c_void_p(d.data_ptr())
    st = S.lib.stmf_masked_error_noalloc(p, p, p, p, 8192, 8256, 2, p, None, None)
    assert st == S.STMF_ENOMEM
