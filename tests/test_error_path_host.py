"""Host-side error path of the C ABI (no device needed): a flush on a machine
without a HIP device fails with OOC_E_DEVICE, the context is failed from then
on (OOC_E_FAILED, message kept), and ooc_destroy still succeeds."""
import pytest

from paper_1709_02125_amd import ooc
from paper_1709_02125_amd.ooc import Const, WRITE, dat

K_FILL = 2


def _no_device():
    import torch
    return torch.cuda.device_count() == 0


@pytest.mark.skipif(not _no_device(), reason="needs a machine without a HIP device")
def test_flush_without_device_fails_the_context():
    c = ooc.Context(2, (8, 8), 1, 1 << 20, 0, bind=False)
    f = c.decl_field("a")
    c.par_loop(K_FILL, ((0, 8), (0, 8)), [dat(f, WRITE), Const(1.0)])
    with pytest.raises(ooc.OocError) as e:
        c.execute()
    assert e.value.code == ooc.E_DEVICE
    for call in (c.execute, lambda: c.reduce(0), lambda: c.set_flags(ooc.FLAG_CYCLIC, 0),
                 lambda: c.debug_fail_after(3)):
        with pytest.raises(ooc.OocError) as e:
            call()
        assert e.value.code in (ooc.E_FAILED, ooc.E_ARG)
    with pytest.raises(ooc.OocError) as e:
        c.execute()
    assert e.value.code == ooc.E_FAILED and "no HIP device" in str(e.value)
    c.close()


def test_fail_after_rejects_a_negative_count():
    c = ooc.Context(2, (8, 8), 1, 1 << 20, 0, bind=False)
    with pytest.raises(ooc.OocError) as e:
        c.debug_fail_after(-1)
    assert e.value.code == ooc.E_ARG
    c.debug_fail_after(0)
    c.close()
