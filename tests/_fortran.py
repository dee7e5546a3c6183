"""Test helpers: Fortran unformatted sequential records written and read in
plain Python (struct), independently of the library's C++ reader and writer.
Layouts: the H.DAT target and symmetry records and the OMEGA records of the
PSTGF paper's sections "Input files" and "Output files"."""
import struct

import numpy as np


def record(payload: bytes, big: bool = False, split: int = 0) -> bytes:
    """One record; with split > 0 it is cut into subrecords of at most `split`
    bytes, marked the way gfortran marks records over 2 GiB (negative head
    markers on all but the last subrecord, negative tail markers on all but
    the first)."""
    e = ">" if big else "<"
    if not split or len(payload) <= split:
        m = struct.pack(e + "i", len(payload))
        return m + payload + m
    parts = [payload[i:i + split] for i in range(0, len(payload), split)]
    out = b""
    for k, p in enumerate(parts):
        head = len(p) if k == len(parts) - 1 else -len(p)
        tail = len(p) if k == 0 else -len(p)
        out += struct.pack(e + "i", head) + p + struct.pack(e + "i", tail)
    return out


def i4(vals, big=False):
    return np.asarray(vals, dtype=(">" if big else "<") + "i4").tobytes()


def r8(vals, big=False):
    return np.asarray(vals, dtype=(">" if big else "<") + "f8").tobytes()


def hdat_target(nelc, nz, lrang2, lamax, enat, lat, isat, ra, bsto, coeff, butt, big=False):
    """Target records of H.DAT / H.DAT000; butt: list of (ebutd, cbutd) per L."""
    nast = len(enat)
    out = record(i4([nelc, nz, lrang2, lamax, nast], big) + r8([ra, bsto], big), big)
    out += record(r8(enat, big), big) + record(i4(lat, big), big) + record(i4(isat, big), big)
    out += record(r8(np.asarray(coeff).reshape(-1), big), big)
    for eb, cb in butt:
        out += record(i4([len(eb)], big), big) + record(r8(eb, big), big) + record(r8(cb, big), big)
    return out


def hdat_symmetry(lrgl2, nspn2, npty2, nconat, l2p, cf, value, wmat, more2=0, big=False, split=0):
    """Symmetry records; cf [lamax][nchan][nchan] is written with its last two
    indices I, N and the multipole index M outermost, i.e. CF(I,N,M) with I
    fastest; wmat [mnp2][nchan] pole by pole."""
    nchan, mnp2 = len(l2p), len(value)
    out = record(i4([lrgl2, nspn2, npty2, nchan, mnp2, more2], big), big)
    out += record(i4(nconat, big), big) + record(i4(l2p, big), big)
    cfm = np.asarray(cf)  # [M][N][I] in memory, so I varies fastest
    out += record(r8(cfm.reshape(-1), big), big, split)
    out += record(r8(value, big), big, split) + record(r8(np.asarray(wmat).reshape(-1), big), big, split)
    return out


def read_records(data: bytes, big: bool = False):
    e = ">" if big else "<"
    pos, out = 0, []
    while pos < len(data):
        buf = b""
        while True:
            (head,) = struct.unpack_from(e + "i", data, pos)
            n = abs(head)
            buf += data[pos + 4:pos + 4 + n]
            pos += 8 + n
            if head >= 0:
                break
        out.append(buf)
    return out
