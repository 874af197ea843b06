"""Pins of the oracle's record layout (AoS offsets, stride) against the C
compiler itself and numpy's independent implementation of C alignment.

The paper's AoS is a C/C++ struct (Section 1, Listing 1; Section 2,
Listing 4), so a real compiler's offsetof/sizeof is the definition.
"""
import fractions
import os
import subprocess

import numpy as np
import pytest

from synth_inputs import BASE_FIELDS, WIDE_FIELDS, particle_size_fields

CTYPE = {"i8": "int8_t", "u8": "uint8_t", "i32": "int32_t", "i64": "int64_t",
         "f32": "float", "f64": "double"}
NPT = {"i8": "i1", "u8": "u1", "i32": "<i4", "i64": "<i8", "f32": "<f4", "f64": "<f8"}

SCHEMAS = {
    "base": BASE_FIELDS,
    "wide": WIDE_FIELDS,
    "listing1": [("id", "i32", 1), ("position", "f64", 1), ("mass", "f32", 1)],
    "usage": [("id", "i32", 1), ("pos", "f64", 3), ("vel", "f64", 3), ("mass", "f32", 1)],
    "particle0": particle_size_fields(0),
    "particle5": particle_size_fields(5),
    "bytes": [("a", "u8", 1), ("b", "i64", 1), ("c", "i8", 3), ("d", "f32", 2), ("e", "u8", 1)],
}


def _c_program(schemas, tmp_path):
    lines = ["#include <stdio.h>", "#include <stdint.h>", "#include <stddef.h>"]
    body = []
    for key, fields in schemas.items():
        for packed in (0, 1):
            attr = " __attribute__((packed))" if packed else ""
            members = " ".join(f"{CTYPE[t]} {n}[{d}];" for n, t, d in fields)
            lines.append(f"struct{attr} S_{key}_{packed} {{ {members} }};")
            offs = ", ".join(f"(long)offsetof(struct S_{key}_{packed}, {n})" for n, _, _ in fields)
            fmt = " ".join(["%ld"] * (len(fields) + 1))
            body.append(f'printf("{key} {packed} {fmt}\\n", (long)sizeof(struct S_{key}_{packed}), {offs});')
    lines.append("int main(void) {")
    lines += body
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-O0", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.strip().splitlines():
        parts = line.split()
        res[(parts[0], int(parts[1]))] = (int(parts[2]), [int(x) for x in parts[3:]])
    return res


@pytest.fixture(scope="module")
def compiled(tmp_path_factory):
    return _c_program(SCHEMAS, tmp_path_factory.mktemp("layout"))


@pytest.mark.parametrize("key", sorted(SCHEMAS))
@pytest.mark.parametrize("packed", [0, 1])
def test_layout_matches_c_compiler(ref, compiled, key, packed):
    offs, stride = ref.Schema(SCHEMAS[key], packed=packed).layout()
    c_size, c_offs = compiled[(key, packed)]
    assert offs == c_offs
    assert stride == c_size


@pytest.mark.parametrize("key", sorted(SCHEMAS))
@pytest.mark.parametrize("packed", [0, 1])
def test_layout_matches_numpy_struct(ref, key, packed):
    fields = SCHEMAS[key]
    dt = np.dtype([(n, NPT[t], (d,)) if d > 1 else (n, NPT[t]) for n, t, d in fields],
                  align=not packed)
    offs, stride = ref.Schema(fields, packed=packed).layout()
    assert offs == [dt.fields[n][1] for n, _, _ in fields]
    assert stride == dt.itemsize


def test_known_strides(ref):
    # natural: base {id@0, pos@8, vel@32} 48 B; wide 80 B; packed 40 / 69 B
    assert ref.Schema(BASE_FIELDS).layout() == ([0, 8, 32], 48)
    assert ref.Schema(BASE_FIELDS, packed=True).layout() == ([0, 4, 28], 40)
    assert ref.Schema(WIDE_FIELDS).layout() == ([0, 8, 16, 40, 52, 64, 72], 80)
    assert ref.Schema(WIDE_FIELDS, packed=True).layout()[1] == 69


def test_paper_record_sizes(ref):
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_record_sizes.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert rows
    for size, nbytes, frac in rows:
        _, stride = ref.Schema(particle_size_fields(int(size))).layout()
        assert stride == int(nbytes)
        assert fractions.Fraction(4, stride) == fractions.Fraction(frac)


def test_bad_schema_rejected(ref):
    with pytest.raises(ValueError):
        ref.Schema([("x", "f64", 4)]).layout()
    with pytest.raises(ValueError):
        ref.Schema([("x", "f64", 0)]).layout()
