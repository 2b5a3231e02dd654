"""A hand-assembled edit stream with Huffman-coded symbols (the stream format
of Sec. 3.3 as the library and the oracle write it), shared by the oracle's
and the device decoder's tests."""
import struct


def huffman_stream(chunk_starts, lengths=(1, 2, 3, 3)):
    """Four particles, 0 and 3 flagged, m = 8; Huffman over the symbols
    3, 7, 9, 200 with lengths 1, 2, 3, 3, so the canonical codes (by length,
    then symbol) are 0, 10, 110, 111.  Symbols x: 3 7, y: 9 200, z: 3 3 give
    the bits 0 10 110 111 0 0 (11 bits); chunks of 4 symbols start at bits 0
    and 9."""
    n, m, xi = 4, 8, 0.25
    step, offset = 4 * xi / (2 ** m - 1), 2 * xi
    bits = [0, 1, 0, 1, 1, 0, 1, 1, 1, 0, 0]
    packed = bytearray(2)
    for q, v in enumerate(bits):
        packed[q // 8] |= v << (q % 8)
    assert bytes(packed) == bytes([218, 1])
    payload = (bytes([0b1001]) + struct.pack("<I", 4) + struct.pack("<4I", 3, 7, 9, 200)
               + bytes(lengths) + struct.pack("<QII", len(bits), 4, 0)
               + struct.pack("<%dQ" % len(chunk_starts), *chunk_starts) + bytes(packed))
    hdr = struct.pack("<IHBBQQddQQII", 0x45434350, 2, m, 2, n, 2, step, offset,
                      len(payload), len(payload), 8, 0)
    codes = {0: [3, 7], 1: [9, 200], 2: [3, 3]}
    return hdr + payload, step, offset, codes
