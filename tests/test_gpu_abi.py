"""The C ABI's scratch convention on the device: a hot call on a ctx whose scratch was
not sized for the batch returns SMPPI_ERR_SHAPE before enqueueing anything (it never
allocates); after smppi_reserve_batch the same call runs."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2302_11719_amd import _lib as L
from paper_2302_11719_amd import core
from paper_2302_11719_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_hot_calls_need_a_reserved_scratch():
    c = core.Context(0)
    p = W.round_to_f32(W.config1(K=300, T=20))
    M, C = W.params_f32(W.MODEL, W.COST)
    db = core.DeviceBatch([p], dtype=torch.float32)
    w = torch.full((db.sum_K,), 1.0 / db.sum_K, device="cuda")
    out = torch.full((2 * db.sum_T,), -5.0, device="cuda")
    args = (c.h, ctypes.byref(db.batch), ctypes.byref(L.model_struct(M)), ctypes.byref(L.cost_struct(C)),
            ctypes.byref(L.Noise(1, 0)), core._p(db.V), core._p(w), core._p(db.iter), core._p(out),
            ctypes.c_void_p(core._stream()))
    print("update on an unreserved ctx", flush=True)
    st = L.lib().smppi_update(*args)
    assert st == 2
    assert b"smppi_reserve_batch" in L.lib().smppi_last_error(c.h)
    torch.cuda.synchronize()
    assert torch.all(out == -5.0)  # nothing ran
    assert L.lib().smppi_reserve_batch(c.h, ctypes.byref(db.batch)) == 0
    assert L.lib().smppi_update(*args) == 0
    torch.cuda.synchronize()
    ref = core.update(c, db, M, C, 1, w)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    # a batch with larger declared bounds than the reservation (which keeps some headroom)
    # is refused again, before anything is launched
    db.batch.k_max = 1 << 24
    assert L.lib().smppi_update(*args) == 2
    db.batch.k_max = db.k_max
    c.close()
