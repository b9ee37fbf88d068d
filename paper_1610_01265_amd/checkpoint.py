"""Checkpoint and resume of a run: device fields (temperature, velocities,
iterates) and networks (master weights, Adam moments and step count,
scalings), in one file.  Written with torch.save and read back with
torch.load(weights_only=True): the file holds tensors, numbers and strings
only, so loading it executes nothing.  A network restored from a checkpoint
continues training exactly as the one it was saved from (cnn_set_state)."""
from __future__ import annotations

import os

import numpy as np
import torch

FORMAT = 1


def save(path, fields=None, nets=None, extra=None) -> None:
    """fields: {name: tensor} (copied to host); nets: {name: Cnn or CnnPC};
    extra: {name: int | float | str | bool}.  The file is replaced
    atomically (written beside it, then renamed)."""
    blob = {"format": FORMAT, "fields": {}, "nets": {}, "extra": {}}
    for k, t in (fields or {}).items():
        blob["fields"][k] = t.detach().to("cpu").clone()
    for k, net in (nets or {}).items():
        st = net.get_state()
        blob["nets"][k] = {"buf": torch.from_numpy(np.ascontiguousarray(st["buf"])),
                           "meta": torch.from_numpy(np.ascontiguousarray(st["meta"]))}
    for k, v in (extra or {}).items():
        if not isinstance(v, (int, float, str, bool)):
            raise TypeError(f"extra[{k!r}] must be a number, string or bool")
        blob["extra"][k] = v
    tmp = f"{path}.tmp"
    torch.save(blob, tmp)
    os.replace(tmp, path)


def load(path, nets=None, device="cuda"):
    """Returns (fields on `device`, extra); restores each network in `nets`
    ({name: Cnn or CnnPC} of the saved shapes) from its saved state."""
    blob = torch.load(path, map_location="cpu", weights_only=True)
    if not isinstance(blob, dict) or blob.get("format") != FORMAT:
        raise ValueError(f"{path}: not a checkpoint of format {FORMAT}")
    fields = {k: t.to(device) for k, t in blob["fields"].items()}
    for k, net in (nets or {}).items():
        if k not in blob["nets"]:
            raise KeyError(f"{path}: no network {k!r}")
        st = blob["nets"][k]
        net.set_state({"buf": st["buf"].numpy(), "meta": st["meta"].numpy()})
    return fields, dict(blob["extra"])
