"""The write-pattern probe of the binning (rambo_roofline_append): it writes
exactly the words it reports, each once, inside the chunks it describes, and
rejects a buffer too small for one run."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

from paper_1910_02611_amd.rambo import EINVAL, lib

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("misaligned", [0, 1])
@pytest.mark.parametrize("streams,run,nwg", [(4, 16, 2), (7, 16, 3), (3, 5, 1)])
def test_append_writes_what_it_reports(misaligned, streams, run, nwg):
    L = lib()
    words = 1 << 16
    buf = torch.full((words,), -1, dtype=torch.int32, device="cuda")
    written = ctypes.c_uint64(0)
    rc = L.rambo_roofline_append(buf.data_ptr(), words, streams, run, misaligned, nwg, ctypes.byref(written),
                                 torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    cap = words // (streams * nwg) // 16 * 16
    rounds = (cap - 15) // run
    assert written.value == rounds * run * streams * nwg
    got = buf.cpu().numpy().view(np.uint32)
    touched = got != 0xFFFFFFFF
    assert int(touched.sum()) == written.value
    # every chunk holds `rounds * run` consecutive words, starting 0..15 words
    # in (at 0 when aligned), and nothing lies past the last chunk
    assert not touched[streams * nwg * cap:].any()
    for c in range(streams * nwg):
        idx = np.flatnonzero(touched[c * cap:(c + 1) * cap])
        assert idx.size == rounds * run
        assert idx[-1] - idx[0] + 1 == rounds * run
        assert idx[0] < 16 and (misaligned or idx[0] == 0)


def test_append_rejects_a_small_buffer():
    L = lib()
    buf = torch.empty(64, dtype=torch.int32, device="cuda")
    written = ctypes.c_uint64(0)
    rc = L.rambo_roofline_append(buf.data_ptr(), 64, 4, 16, 1, 2, ctypes.byref(written),
                                 torch.cuda.current_stream().cuda_stream)
    assert rc == EINVAL

