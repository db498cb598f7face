"""Offline storage of packed fields, host side (no device access): the
header is read and checked before any copy, so malformed or mismatching
files are rejected here."""
import struct

import pytest

from paper_2302_09224_amd import hisq

HDR = struct.Struct("<8s i i 4i q i i 3d Q Q Q 32x")   # the documented 128-byte header


def header(kind=1, fmt=3, dims=(0, 0, 0, 0), nsites=100, recon=0, scales=(0.0, 0.0, 0.0), b0=None, b1=0, ck=0,
           magic=b"HISQPK01"):
    if b0 is None:
        b0 = nsites * hisq.SPINOR_BYTES[fmt]
    return HDR.pack(magic, kind, fmt, *dims, nsites, recon, 0, *scales, b0, b1, ck)


@pytest.fixture(scope="module")
def lib():
    return hisq.load()


def test_header_size():
    assert HDR.size == 128


def test_field_info_reads_spinor_and_gauge_headers(lib, tmp_path):
    p = tmp_path / "s.hisq"
    p.write_bytes(header(fmt=hisq.SPINOR_INT24, nsites=77) + bytes(77 * 20))
    info = hisq.field_info(str(p))
    assert info["kind"] == hisq.FIELD_SPINOR and info["fmt"] == hisq.SPINOR_INT24
    assert info["nsites"] == 77 and info["bytes0"] == 77 * 20 and info["bytes1"] == 0
    dims = (4, 4, 6, 8)
    b0 = hisq.hisq_gauge_bytes(dims, hisq.GAUGE_FIX16)
    b1 = hisq.hisq_gauge_long_bytes(dims, hisq.GAUGE_FIX16, 12)
    g = tmp_path / "g.hisq"
    g.write_bytes(header(kind=2, fmt=hisq.GAUGE_FIX16, dims=dims, nsites=4 * 4 * 6 * 8, recon=12,
                         scales=(1.0, 1.0, -1 / 24), b0=b0, b1=b1))
    info = hisq.field_info(str(g))
    assert info["kind"] == hisq.FIELD_GAUGE and info["dims"] == dims and info["long_recon"] == 12
    assert (info["bytes0"], info["bytes1"]) == (b0, b1)


@pytest.mark.parametrize("case", ["missing", "short", "magic", "kind", "spinor_size", "spinor_fmt", "gauge_dims",
                                  "gauge_recon", "gauge_size"])
def test_malformed_files_are_eio(lib, tmp_path, case):
    p = tmp_path / "bad.hisq"
    dims = (4, 4, 4, 4)
    gb0, gb1 = hisq.hisq_gauge_bytes(dims, 3), hisq.hisq_gauge_long_bytes(dims, 3, 18)
    data = {
        "short": header()[:100],
        "magic": header(magic=b"HISQPK02"),
        "kind": header(kind=3),
        "spinor_size": header(b0=1600 + 16),
        "spinor_fmt": header(fmt=6, b0=0),
        "gauge_dims": header(kind=2, fmt=3, dims=(4, 4, 4, 5), recon=18, b0=gb0, b1=gb1),
        "gauge_recon": header(kind=2, fmt=3, dims=dims, recon=8, b0=gb0, b1=gb1),
        "gauge_size": header(kind=2, fmt=3, dims=dims, recon=18, b0=gb0, b1=gb1 + 16),
    }
    if case != "missing":
        p.write_bytes(data[case])
    with pytest.raises(hisq.HisqError) as e:
        hisq.field_info(str(p))
    assert e.value.status == -8


def test_load_rejects_other_kind_format_or_size(lib, tmp_path):
    p = tmp_path / "s.hisq"
    p.write_bytes(header(fmt=hisq.SPINOR_INT20, nsites=64) + bytes(64 * 16))
    fake = 1 << 20                       # never dereferenced: the header check fails first
    assert lib.hisq_spinor_load(str(p).encode(), fake, 64, hisq.SPINOR_HALF16, None) == -1
    assert lib.hisq_spinor_load(str(p).encode(), fake, 65, hisq.SPINOR_INT20, None) == -1
    assert lib.hisq_spinor_load(str(p).encode(), None, 64, hisq.SPINOR_INT20, None) == -1
    g = hisq.hisq_gauge()
    assert lib.hisq_gauge_load(str(p).encode(), g, fake, 1 << 30, fake, 1 << 30, None) == -1   # a spinor file
    assert lib.hisq_gauge_load(str(p).encode(), g, fake + 8, 1 << 30, fake, 1 << 30, None) == -2  # unaligned
    dims = (4, 4, 4, 4)
    gb0, gb1 = hisq.hisq_gauge_bytes(dims, 2), hisq.hisq_gauge_long_bytes(dims, 2, 12)
    q = tmp_path / "g.hisq"
    q.write_bytes(header(kind=2, fmt=2, dims=dims, nsites=256, recon=12, b0=gb0, b1=gb1))
    assert lib.hisq_gauge_load(str(q).encode(), g, fake, gb0 - 16, fake, gb1, None) == -1       # buffer too small
    assert lib.hisq_spinor_save(str(q).encode(), fake, 10, 9, None) == -1                       # unknown format
