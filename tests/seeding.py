"""Stable seeds for test case generators.

Python's hash() of a str (and of a tuple holding one) changes from process to
process, so seeds are taken from a CRC-32 of the parts' repr instead: the same
cases are drawn in every run.
"""
import zlib


def seed(*parts) -> int:
    return zlib.crc32(repr(parts).encode())
