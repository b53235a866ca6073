"""MLP checkpoint round trip on the host (plain arrays, nothing unpickled)."""
import numpy as np
import pytest
import torch

from oracle import learned


def test_checkpoint_round_trip(tmp_path):
    import paper_2102_03011_amd as sg
    from paper_2102_03011_amd import train
    m = learned.init_mlp(1, mean=np.arange(8.0), std=np.arange(1.0, 9.0))
    p = sg.MLPParams.from_arrays(m.w1, m.b1, m.w2, m.b2, m.w3, 0.5, m.mean, 1.0 / m.std, device="cpu")
    path = str(tmp_path / "w.npz")
    train.save_mlp(path, p, {"note": "x"})
    q, meta = train.load_mlp(path, device="cpu")
    assert torch.equal(p.w, q.w) and torch.equal(p.b, q.b) and meta["note"] == "x"
    w1, b1, w2, b2, w3, b3 = q.weights_f64()
    assert np.array_equal(w1, learned.bf16_round(m.w1)) and b3 == 0.5
    assert np.allclose(1.0 / q.b[140:148].double().numpy(), m.std, rtol=1e-7)


def test_checkpoint_rejects_other_format(tmp_path):
    from paper_2102_03011_amd import train
    path = str(tmp_path / "bad.npz")
    np.savez(path, w_bf16=np.zeros(4672, np.uint16), b=np.zeros(148, np.float32),
             meta=np.frombuffer(b'{"format": 99}', dtype=np.uint8))
    with pytest.raises(ValueError):
        train.load_mlp(path, device="cpu")
