"""plu_measure_peak through the C ABI: the measured ceilings are positive and
no higher than the datasheet peaks they stand beside (MI355X dense
matrix-core rates, 8 TB/s of HBM), and bad arguments are refused before any
launch."""

import ctypes

import pytest

from tests.gpu_common import torch, have_gpu, handle as make_handle

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

DATASHEET = {0: 157.3, 1: 2500.0, 2: 5000.0, 3: 8000.0}


@pytest.fixture(scope="module")
def handle():
    h = make_handle()
    yield h
    h.close()


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_matrix_core_rates_are_below_the_datasheet(handle, kind):
    r = handle.measure_peak(kind, reps=2)
    assert 0.2 * DATASHEET[kind] < r <= 1.02 * DATASHEET[kind], r


def test_hbm_read_rate_is_below_the_datasheet(handle):
    buf = torch.empty(2 ** 28, dtype=torch.float32, device="cuda:0")
    r = handle.measure_peak(3, buf, reps=2)
    assert 0.2 * DATASHEET[3] < r <= DATASHEET[3], r


def test_bad_arguments_are_refused(handle):
    import paper_2002_07138_amd as plu
    lib = plu.library()
    out = ctypes.c_double(-1.0)
    h = handle._h
    assert lib.plu_measure_peak(h, 4, None, 0, 1, ctypes.byref(out)) == -2
    assert lib.plu_measure_peak(h, 3, None, 1 << 22, 1, ctypes.byref(out)) == -3
    buf = torch.empty(1024, dtype=torch.float32, device="cuda:0")
    assert lib.plu_measure_peak(h, 3, ctypes.c_void_p(buf.data_ptr()), 4096, 1,
                                ctypes.byref(out)) == -4
    assert lib.plu_measure_peak(h, 0, None, 0, 0, ctypes.byref(out)) == -5
    assert lib.plu_measure_peak(h, 0, None, 0, 1, None) == -6
    assert out.value == -1.0
