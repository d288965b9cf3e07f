"""Autotuner of the persistent batched launch: picks the workgroup size, cells per thread and
workgroups per CU by timing short probe runs of the caller's own batch, and caches the choice
per (device, batch size, total cells) in a JSON file.

The probe runs advance copies of the state, so the caller's tensors are untouched.
"""
import json
import os

import torch

from . import api

CANDIDATES = [(64, 2, 0), (64, 4, 0), (128, 2, 0), (128, 4, 0), (256, 1, 0), (256, 2, 0),
              (256, 4, 0), (128, 2, 4), (64, 4, 8)]
CACHE = os.environ.get("WZN_TUNING_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "wenozn", "tuning.json"))


def _key(u, batch):
    name = torch.cuda.get_device_name(u.device).replace(" ", "_")
    total = u.shape[1]
    bucket = 1 << max(0, int(total - 1).bit_length())  # next power of two
    return "%s|batched|B%d|T%d" % (name, batch, bucket)


def _load():
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(db):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(db, fh, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def tune_batched(u, offsets, dx, order=None, probe_steps=3, candidates=CANDIDATES,
                 use_cache=True, log=None):
    """Return (WznBatchTuning, timings) for this batch."""
    batch = offsets.numel() - 1
    key = _key(u, batch)
    db = _load() if use_cache else {}
    if key in db:
        nt, k, bpc = db[key]["choice"]
        return api.batch_tuning(nt, k, bpc), db[key].get("ms", {})
    work = u.clone()
    stage = torch.empty((2,) + tuple(u.shape), dtype=u.dtype, device=u.device)
    timings = {}
    for nt, k, bpc in candidates:
        tn = api.batch_tuning(nt, k, bpc)
        work.copy_(u)
        api.batched_rk3_run_1d(work, offsets, dx, 1, order=order, tuning=tn, stage=stage)
        work.copy_(u)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        api.batched_rk3_run_1d(work, offsets, dx, probe_steps, order=order, tuning=tn,
                               stage=stage)
        e.record()
        torch.cuda.synchronize()
        timings["%d/%d/%d" % (nt, k, bpc)] = s.elapsed_time(e) / probe_steps
        if log:
            log("tune nt=%d k=%d bpc=%d: %.3f ms/step" % (nt, k, bpc, timings["%d/%d/%d" % (nt, k, bpc)]))
    best = min(timings, key=timings.get)
    nt, k, bpc = (int(x) for x in best.split("/"))
    if use_cache:
        db[key] = {"choice": [nt, k, bpc], "ms": timings}
        _store(db)
    return api.batch_tuning(nt, k, bpc), timings
