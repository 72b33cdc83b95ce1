"""The device copy of the blob workload is the host recipe's output."""
import numpy as np

import synth


def test_blob_case_device_matches_host():
    a = synth.blob_case((24, 32, 16), seed=77)
    t, v = synth.blob_case_device((24, 32, 16), 77, device="cpu")
    assert np.abs(a["rhoT"] - t.numpy()).max() == 0.0
    assert np.abs(a["v_true"] - v.numpy()).max() == 0.0
