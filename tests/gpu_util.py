"""Helpers shared by the GPU tests: record packing with numpy structured
dtypes (independent of both the library and the oracle), ulp distances and
periodic distances."""
import numpy as np

import synth_inputs as si

NPT = {"i8": "i1", "u8": "u1", "i32": "<i4", "i64": "<i8", "f32": "<f4", "f64": "<f8"}
L = si.BOX_L


def record_dtype(fields, packed=False):
    return np.dtype([(n, NPT[t], (d,)) if d > 1 else (n, NPT[t]) for n, t, d in fields],
                    align=not packed)


def to_aos(fields, arrays, packed=False):
    """AoS bytes (padding 0) of SoA arrays, packed by numpy's struct rules."""
    n = len(arrays[0])
    rec = np.zeros(n, dtype=record_dtype(fields, packed))
    a = 0
    for name, _, d in fields:
        for c in range(d):
            if d == 1:
                rec[name] = arrays[a]
            else:
                rec[name][:, c] = arrays[a]
            a += 1
    return rec.view(np.uint8).reshape(-1).copy()


def from_aos(fields, buf, n, packed=False):
    rec = np.ascontiguousarray(buf[: n * record_dtype(fields, packed).itemsize]).view(
        record_dtype(fields, packed))
    out = []
    for name, _, d in fields:
        for c in range(d):
            out.append(np.ascontiguousarray(rec[name] if d == 1 else rec[name][:, c]))
    return out


def ulp_distance(a, b):
    """Per-element distance in units in the last place (same dtype)."""
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    it = {np.dtype(np.float32): np.int32, np.dtype(np.float64): np.int64}[a.dtype]
    ia = a.view(it).astype(np.int64)
    ib = b.view(it).astype(np.int64)
    big = np.iinfo(it).min
    ia = np.where(ia < 0, big - ia, ia)
    ib = np.where(ib < 0, big - ib, ib)
    return np.abs(ia - ib)


def pdist(a, b):
    d = np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))
    return np.minimum(d, L - d)


def assert_positions_close(got, want, tol=1e-12 * L):
    """Periodic distance within tol (default 1e-12 of the box edge)."""
    d = pdist(got, want)
    assert d.max() <= tol, f"max periodic distance {d.max():.3e} > {tol:.3e}"


def assert_fields_close(got, want, rel=1e-6):
    """|got - want| <= rel * max(|want|, 1), element by element."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    err = np.abs(got - want) / np.maximum(np.abs(want), 1.0)
    assert err.max() <= rel, f"max scaled error {err.max():.3e} > {rel:.1e}"
