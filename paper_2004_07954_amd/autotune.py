"""Autotuner of the persistent batched launch: picks the workgroup size, cells per thread and
workgroups per CU by timing short probe runs of the caller's own batch, and caches the choice
per (device, batch size, total cells) in a JSON file.

The probe runs advance copies of the state, so the caller's tensors are untouched.
"""
import json
import os

import torch

from . import api

# (threads per workgroup, cells per thread, workgroups per CU (0: occupancy limit), layout)
CANDIDATES = [(64, 2, 0, 0), (64, 4, 0, 0), (128, 2, 0, 0), (128, 4, 0, 0), (256, 1, 0, 0),
              (256, 2, 0, 0), (256, 4, 0, 0), (128, 2, 4, 0), (64, 4, 8, 0), (128, 4, 0, 1),
              (256, 2, 0, 1), (256, 4, 0, 1)]
CACHE = os.environ.get("WZN_TUNING_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "wenozn", "tuning.json"))


def _key(u, batch):
    name = torch.cuda.get_device_name(u.device).replace(" ", "_")
    total = u.shape[1]
    bucket = 1 << max(0, int(total - 1).bit_length())  # next power of two
    return "%s|batched2|B%d|T%d" % (name, batch, bucket)


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
        nt, k, bpc, lay = db[key]["choice"]
        return api.batch_tuning(nt, k, bpc, lay), db[key].get("ms", {})
    work = u.clone()
    stage = torch.empty((2,) + tuple(u.shape), dtype=u.dtype, device=u.device)
    timings = {}
    for nt, k, bpc, lay in candidates:
        tn = api.batch_tuning(nt, k, bpc, lay)
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
        key_t = "%d/%d/%d/%d" % (nt, k, bpc, lay)
        timings[key_t] = s.elapsed_time(e) / probe_steps
        if log:
            log("tune nt=%d k=%d bpc=%d layout=%d: %.3f ms/step" % (nt, k, bpc, lay, timings[key_t]))
    best = min(timings, key=timings.get)
    nt, k, bpc, lay = (int(x) for x in best.split("/"))
    if use_cache:
        db[key] = {"choice": [nt, k, bpc, lay], "ms": timings}
        _store(db)
    return api.batch_tuning(nt, k, bpc, lay), timings


# (threads per workgroup, cells per thread, layout): layouts 0 (both signs staged) and 1 (one
# sign at a time)
ROW_SHAPES = [(256, 4, 0), (256, 2, 0), (256, 1, 0), (128, 4, 0), (128, 8, 0), (64, 8, 0),
              (64, 4, 0), (64, 2, 0), (64, 1, 0), (256, 4, 1), (256, 2, 1), (128, 4, 1), (64, 4, 1)]


def get_row_tuning(nvar, n):
    """(nt, k, layout) the 1D entry points use for nvar components of n cells."""
    import ctypes as C
    from ._lib import check, lib
    nt, k, lay = C.c_int32(), C.c_int32(), C.c_int32()
    check(lib().wzn_get_row_tuning(int(nvar), int(n), C.byref(nt), C.byref(k), C.byref(lay)))
    return nt.value, k.value, lay.value


def set_row_tuning(nt, k, layout=0):
    from ._lib import check, lib
    check(lib().wzn_set_row_tuning(int(nt), int(k), int(layout)))


def tune_rows(n, steps=50, shapes=ROW_SHAPES, log=None, apply=True, rounds=1):
    """Time the 1D Euler TVD-RK3 stage kernel at grid size n for every launch shape on
    Shu-Osher-like data and (optionally) install the fastest process-wide.  With rounds > 1
    the shapes are timed in turn that many times and each keeps its best time, so that a
    clock ramp or a noisy sample does not decide between shapes a few per cent apart.
    Returns ((nt, k, layout), {shape: ms per step})."""
    from . import inputs as I
    u0, dx = I.shu_osher_like(n)
    base = torch.tensor(u0, dtype=torch.float64, device="cuda")
    u = base.clone()
    stage = torch.empty((2,) + tuple(u.shape), dtype=torch.float64, device="cuda")
    prm = api.params("euler")
    timings = {}
    for _ in range(max(1, rounds)):
        for nt, k, lay in shapes:
            set_row_tuning(nt, k, lay)
            u.copy_(base)
            api.rk3_run_1d(u, dx, 2, prm=prm, stage=stage)
            u.copy_(base)
            torch.cuda.synchronize()
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            api.rk3_run_1d(u, dx, steps, prm=prm, stage=stage)
            e.record()
            torch.cuda.synchronize()
            key = "%d/%d/%d" % (nt, k, lay)
            t = s.elapsed_time(e) / steps
            timings[key] = min(t, timings.get(key, t))
    if log:
        for key, t in timings.items():
            log("rows n=%d shape %s: %.4f ms/step" % (n, key, t))
    best = min(timings, key=timings.get)
    nt, k, lay = (int(x) for x in best.split("/"))
    set_row_tuning(nt, k, lay) if apply else set_row_tuning(0, 0)
    return (nt, k, lay), timings
