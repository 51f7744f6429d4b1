"""The allocation-free pion correlator (dd_pion_correlator_noalloc): through the C ABI it
gives bitwise the result of dd_pion_correlator (the same kernels, the partial sums in the
static device scratch instead of the context's workspace), on two calls in a row, the second
with a smaller input (fewer columns and another source slice, so stale scratch from the first
call would show), and refuses a request beyond its scratch with DD_ERR_ARG."""
import ctypes as C

import numpy as np
import pytest
import torch

from helpers import lib, step

pytestmark = pytest.mark.gpu


def test_noalloc_pion_correlator_matches_the_workspace_one():
    dd = lib()
    T, L = 16, 8
    step("no-alloc pion correlator")
    ctx = dd.Context(T, L, -1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4100)
    V = T * L ** 3
    S1 = torch.randn((12, 12, V), dtype=torch.complex128, device="cuda", generator=gen)
    S2 = torch.randn((3, 12, V), dtype=torch.complex128, device="cuda", generator=gen)
    for S, t_src in ((S1, 5), (S2, 11)):
        want = dd.pion_correlator(ctx, S, t_src)
        got = dd.pion_correlator_noalloc(ctx, S, t_src)
        assert np.array_equal(got, want), (got - want)
        assert np.all(want > 0)
    # a request beyond the static scratch is refused before any launch
    big = dd.Context(4096, 2, -1)
    Sb = torch.zeros((48, 12, 4096 * 8), dtype=torch.complex128, device="cuda")
    out = (C.c_double * 4096)()
    st = dd._lib.dd_pion_correlator_noalloc(big._h, C.c_void_p(Sb.data_ptr()), 48, 0, out)
    assert st == dd.DD_ERR_ARG
    assert "static scratch" in dd._lib.dd_last_error(big._h).decode()
