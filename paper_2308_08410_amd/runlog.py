"""Run records for long fits and training runs.

* ``RunLog``: a JSON-lines log whose first record describes the run's host (CPU
  model, logical cores), device and library and the run's configuration; every
  later record is one progress line (iteration, losses, time), flushed as written.
* ``save_checkpoint`` / ``load_checkpoint``: named arrays in one ``.npz`` file
  (numpy's format, read back without pickling), written to a temporary name and
  renamed, so a run killed while saving leaves the previous checkpoint intact.
"""
from __future__ import annotations

import json
import os
import platform
import time

import numpy as np


def host_info() -> dict:
    """CPU model, logical core count and host name of the machine this runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(cpu_model=model, nproc=os.cpu_count(), hostname=platform.node(),
                python=platform.python_version())


def device_info() -> dict:
    """The GPU torch sees (name, memory) and the library's version string."""
    out = {}
    try:
        import torch
        if torch.cuda.is_available():
            p = torch.cuda.get_device_properties(0)
            out.update(gpu=p.name, gpu_memory_gb=round(p.total_memory / 2 ** 30, 1), torch=torch.__version__)
    except Exception as e:          # the log must not stop a run
        out["gpu_error"] = repr(e)
    try:
        from . import binding
        out["library"] = binding.version()
    except Exception as e:
        out["library_error"] = repr(e)
    return out


def _plain(v):
    if isinstance(v, dict):
        return {k: _plain(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_plain(x) for x in v]
    if isinstance(v, np.ndarray):
        return v.tolist()
    if isinstance(v, (np.floating, np.integer)):
        return v.item()
    if hasattr(v, "detach"):        # a torch tensor
        return v.detach().cpu().numpy().tolist()
    return v


class RunLog:
    """Append-only JSON-lines log (one JSON object per line)."""

    def __init__(self, path: str, kind: str, config: dict, device: bool = True):
        self.path = path
        self._f = open(path, "a")
        self.t0 = time.time()
        self.write(event="start", kind=kind, host=host_info(), device=device_info() if device else None,
                   config=config)

    def write(self, **record):
        record = dict(time=time.time(), elapsed_s=time.time() - self.t0, **record)
        self._f.write(json.dumps(_plain(record)) + "\n")
        self._f.flush()

    def close(self, **record):
        if self._f:
            self.write(event="end", **record)
            self._f.close()
            self._f = None


def read_log(path: str) -> list:
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]


def save_checkpoint(path: str, **arrays):
    """Write the named arrays (numpy arrays, scalars or torch tensors) to `path`."""
    data = {}
    for k, v in arrays.items():
        if hasattr(v, "detach"):
            v = v.detach().cpu().numpy()
        data[k] = np.asarray(v)
        if data[k].dtype == object:
            raise TypeError(f"checkpoint entry {k!r} is not a plain array")
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, **data)
    os.replace(tmp, path)


def load_checkpoint(path: str) -> dict:
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}
