"""pic_probe_lds_atomics, the measurement of the deposition's LDS-atomic bound: finite rates within what
64-lane compute units at ~2.4 GHz can issue, and its argument checks."""

import pytest

from gpu_common import banner

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2106_12919_amd import lib as piclib  # noqa: E402


def test_lds_atomic_probe_rates():
    banner("LDS atomic probe")
    torch.cuda.set_device(0)
    for bits in (32, 64):
        r = piclib.pic_probe_lds_atomics(bits, 4096)
        per_clock = r / 2.4e9
        print(f"{bits}-bit LDS atomics: {per_clock:.2f} lane-ops per clock per CU")
        assert 0.5 <= per_clock <= 128.0
    with pytest.raises(RuntimeError):
        piclib.pic_probe_lds_atomics(16, 4096)
    with pytest.raises(RuntimeError):
        piclib.pic_probe_lds_atomics(32, 1000)
