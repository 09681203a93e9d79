"""The Python binding keeps the buffers that a batch launch writes alive: a
view record holds its framebuffer and image tensors, and launches hold them
until the event recorded after the launch has completed (CPU only: tensors on
the host, a stand-in event)."""
import gc
import weakref

import numpy as np
import torch

from paper_2104_07526_amd import pcr


def test_view_record_holds_its_buffers():
    W, H = 8, 4
    fb = torch.empty(pcr.fb_bytes(W, H, pcr.BASIC) // 8, dtype=torch.int64)
    img = torch.empty(W * H, dtype=torch.int32)
    rf, ri = weakref.ref(fb), weakref.ref(img)
    v = pcr.make_view(np.eye(4), W, H, pcr.BASIC, fb, img)
    del fb, img
    gc.collect()
    assert rf() is not None and ri() is not None
    assert v.fb == rf().data_ptr() and v.rgba_out == ri().data_ptr()
    del v
    gc.collect()
    assert rf() is None and ri() is None


class FakeEvent:
    def __init__(self):
        self.done = False

    def query(self):
        return self.done


def test_launch_holds_buffers_until_completion():
    W, H = 8, 4
    held = pcr._InFlight()
    fb = torch.empty(pcr.fb_bytes(W, H, pcr.HQ) // 8, dtype=torch.int64)
    img = torch.empty(W * H, dtype=torch.int32)
    rf = weakref.ref(fb)
    views = [pcr.make_view(np.eye(4), W, H, pcr.HQ, fb, img)]
    ev = FakeEvent()
    held.hold(ev, pcr._held_refs(None, views))
    del fb, img, views
    gc.collect()
    assert rf() is not None and held.pending() == 1     # launch not complete: still held
    ev.done = True
    assert held.pending() == 0                          # completed: released
    gc.collect()
    assert rf() is None
