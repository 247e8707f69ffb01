"""Persistent cache of tuned stage groupings.

The library keeps plans (which radix-K passes share a launch) per field
object and process; ``gfp_tune`` measures and stores them there.  This module
tunes a set of keys and saves / restores the chosen plan strings as JSON,
keyed by GPU architecture, field (k, r), transform size, batch class and
layout, so a later process can apply them with ``gfp_plan_set`` instead of
tuning again.  Plans never change results, only speed.

    entries = tune(field, sizes=[4096, 2 ** 20], nvecs=[1, 2, 16])
    save("plans.json", field, entries, arch="gfx950")
    ...
    load("plans.json", other_field, arch="gfx950")
"""

from __future__ import annotations

import json
import os

from .gfp import LAYOUT_DIGIT_MAJOR, LAYOUT_ELEMENT_MAJOR

FORMAT = 1


def batch_class(nvec: int) -> int:
    """The library's batch classes: 1, 2-7, 8-63, 64 and more transforms."""
    return 0 if nvec <= 1 else 1 if nvec < 8 else 2 if nvec < 64 else 3


_CLASS_REP = {0: 1, 1: 2, 2: 8, 3: 64}  # a transform count inside each class


def field_key(field, arch: str) -> str:
    return "%s|k=%d|r=%d" % (arch, field.k, field.r)


def _entry_key(n: int, cls: int, layout: int) -> str:
    return "%d|%d|%d" % (n, cls, layout)


def tune(field, sizes, nvecs=(1,), layouts=(LAYOUT_DIGIT_MAJOR, LAYOUT_ELEMENT_MAJOR), stream=None) -> dict:
    """Run the library's tuner for every (size, transform count, layout) and
    return {entry key: plan}."""
    out = {}
    for n in sizes:
        for nv in nvecs:
            for lay in layouts:
                plan, _ = field.tune(n, nvec=nv, layout=lay, stream=stream)
                out[_entry_key(n, batch_class(nv), lay)] = plan
    return out


def export_plans(field, keys) -> dict:
    """Current plans (tuned, set or default) of (n, nvec, layout) keys."""
    return {_entry_key(n, batch_class(nv), lay): field.plan(n, nvec=nv, layout=lay) for n, nv, lay in keys}


def apply(field, entries: dict) -> int:
    """Set every plan of {entry key: plan}; returns how many were set."""
    count = 0
    for key, plan in entries.items():
        n, cls, lay = (int(v) for v in key.split("|"))
        field.set_plan(n, plan, nvec=_CLASS_REP[cls], layout=lay)
        count += 1
    return count


def save(path: str, field, entries: dict, arch: str):
    """Merge entries into the JSON cache at path under this field and arch."""
    data = {"format": FORMAT, "fields": {}}
    if os.path.exists(path):
        with open(path) as fh:
            old = json.load(fh)
        if old.get("format") == FORMAT:
            data = old
    data["fields"].setdefault(field_key(field, arch), {}).update(entries)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load(path: str, field, arch: str) -> int:
    """Apply the cached plans of this field and arch; returns how many."""
    if not os.path.exists(path):
        return 0
    with open(path) as fh:
        data = json.load(fh)
    if data.get("format") != FORMAT:
        return 0
    return apply(field, data.get("fields", {}).get(field_key(field, arch), {}))
