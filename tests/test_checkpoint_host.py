"""The checkpoint file format on the host: fields, network states and
extra values survive a save / load round trip exactly, the file is read with
the safe loader only, and bad inputs are refused."""
import numpy as np
import pytest
import torch

from paper_1610_01265_amd import checkpoint


class _FakeNet:
    def __init__(self, buf, meta):
        self.state = {"buf": buf, "meta": meta}

    def get_state(self):
        return self.state

    def set_state(self, state):
        self.state = {"buf": np.array(state["buf"]), "meta": np.array(state["meta"])}


def test_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    T = torch.from_numpy(rng.standard_normal((3, 4, 5)))
    net = _FakeNet(rng.standard_normal(30).astype(np.float32), rng.standard_normal(8))
    path = str(tmp_path / "run.pt")
    checkpoint.save(path, fields={"T": T}, nets={"guess": net}, extra={"step": 7, "dt": 0.5})
    other = _FakeNet(np.zeros(30, np.float32), np.zeros(8))
    fields, extra = checkpoint.load(path, nets={"guess": other}, device="cpu")
    assert torch.equal(fields["T"], T) and fields["T"].dtype == torch.float64
    assert np.array_equal(other.state["buf"], net.state["buf"])
    assert np.array_equal(other.state["meta"], net.state["meta"])
    assert extra == {"step": 7, "dt": 0.5}
    # the file is plain tensors and containers: the safe loader reads it
    blob = torch.load(path, weights_only=True)
    assert blob["format"] == checkpoint.FORMAT


def test_refusals(tmp_path):
    path = str(tmp_path / "bad.pt")
    with pytest.raises(TypeError):
        checkpoint.save(path, extra={"obj": object()})
    torch.save({"format": 99}, path)
    with pytest.raises(ValueError):
        checkpoint.load(path, device="cpu")
    checkpoint.save(path)
    with pytest.raises(KeyError):
        checkpoint.load(path, nets={"missing": _FakeNet(None, None)}, device="cpu")
