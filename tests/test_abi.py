"""The C-ABI library loads and exports every entry point that
include/rmhd.h declares; argument checks reject bad descriptors on the host
(no device needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "rmhd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rmhd_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("rmhd_init_grid", "rmhd_set_metric", "rmhd_imex_stage", "rmhd_con2prim", "rmhd_step",
              "rmhd_prim2con", "rmhd_max_signal_speed", "rmhd_failures", "rmhd_destroy", "rmhd_last_error",
              "rmhd_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2510_18968_amd import rmhd
    L = C.CDLL(rmhd.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(rmhd.SYMBOLS) <= set(declared())


def test_descriptor_validation_on_host():
    from paper_2510_18968_amd import rmhd
    L = rmhd.lib()
    good = rmhd.make_desc((16, 16, 16), 7, (0.1,) * 3, (0, 0, 0), 2.0)
    assert L.rmhd_workspace_bytes(C.byref(good)) > 0
    for field, value in (("ng", 2), ("recon", 7), ("gamma_ad", 1.0), ("active_mask", 0), ("c2p_maxit", 0)):
        d = rmhd.make_desc((16, 16, 16), 7, (0.1,) * 3, (0, 0, 0), 2.0)
        setattr(d, field, value)
        assert L.rmhd_workspace_bytes(C.byref(d)) == 0
        assert L.rmhd_last_error().decode()
    d = rmhd.make_desc((2, 16, 16), 7, (0.1,) * 3, (0, 0, 0), 2.0)     # too few cells on an active axis
    assert L.rmhd_workspace_bytes(C.byref(d)) == 0
    ctx = C.c_void_p()
    assert L.rmhd_init_grid(C.byref(good), None, 0, None, C.byref(ctx)) == -1
    assert "workspace" in L.rmhd_last_error().decode()


@pytest.mark.parametrize("n,active,x_align", [((16, 16, 16), 7, 0), ((256, 256, 256), 7, 1), ((20, 12, 1), 3, 1),
                                              ((2048, 64, 1), 1, 1), ((400, 1, 1), 1, 0)])
def test_padded_extent_and_layout_round_trip(n, active, x_align):
    """The library's padded extents follow the documented layout (3 cells of
    padding per side on active axes, 16 along x with x_align), and an array
    of the 3-ghost layout survives the trip into the grid's layout and back."""
    import numpy as np
    import torch
    from paper_2510_18968_amd import rmhd
    d = rmhd.make_desc(n, active, (0.1,) * 3, (1, 1, 1), 2.0, x_align=x_align)
    pads = [((16 if (k == 0 and x_align) else 3) if (active >> k) & 1 else 0) for k in range(3)]
    ext = rmhd.padded_extent(d)
    assert ext == tuple(n[k] + 2 * pads[k] for k in (2, 1, 0))
    if x_align:
        assert ext[2] % 16 == 0 or n[0] % 16 != 0          # aligned rows when n_x is a multiple of 16
    ws = rmhd.lib().rmhd_workspace_bytes(C.byref(d))
    assert ws >= 14 * 8 * int(np.prod(ext))
    if np.prod(ext) > 4e6:
        return
    std = tuple(n[k] + 2 * (3 if (active >> k) & 1 else 0) for k in (2, 1, 0))
    a = torch.from_numpy(np.random.default_rng(3).standard_normal((2,) + std))
    t = rmhd.to_layout(a, d)
    assert tuple(t.shape[1:]) == ext
    assert torch.equal(rmhd.from_layout(t, d), a)
    assert float(t.abs().sum()) == float(a.abs().sum())    # the extra padding is zero
