"""Counter-based random numbers written with plain torch int64 ops.

The generator is SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the i-th output of a stream
with state s is mix64(s + (i + 1) * GOLDEN).  Because every draw is a pure
function of (seed, stream, index), the same code yields the same bytes on
the CPU and on a GPU, and any subset of a matrix can be regenerated on its
own.  torch int64 arithmetic wraps modulo 2**64, which is the unsigned
arithmetic SplitMix64 is defined in; right shifts are made logical by
masking.

This module holds no SpGEMM arithmetic; it only draws numbers.
"""
from __future__ import annotations

import torch

_U64 = 1 << 64


def _s64(x: int) -> int:
    """Map an unsigned 64-bit constant to the int64 with the same bits."""
    x &= _U64 - 1
    return x - _U64 if x >= (1 << 63) else x


GOLDEN = _s64(0x9E3779B97F4A7C15)
_M1 = _s64(0xBF58476D1CE4E5B9)
_M2 = _s64(0x94D049BB133111EB)


def _srl(z: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 bits."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def mix64(z: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output function (the published constants 30/27/31)."""
    z = (z ^ _srl(z, 30)) * _M1
    z = (z ^ _srl(z, 27)) * _M2
    return z ^ _srl(z, 31)


def mix64_int(z: int) -> int:
    """Python-int twin of mix64, used only to derive stream states."""
    z &= _U64 - 1
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & (_U64 - 1)
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & (_U64 - 1)
    return z ^ (z >> 31)


class Stream:
    """One SplitMix64 stream, addressed by an int64 counter.

    ``Stream(seed, tag)`` derives its state from the seed and a small
    integer tag so that independent quantities (row draws, value draws,
    target draws, ...) never share counters.
    """

    def __init__(self, seed: int, tag: int):
        self.state = _s64(mix64_int(mix64_int(seed) ^ ((tag * 0x632BE59BD9B4E019) & (_U64 - 1))))
        self._first = _s64(self.state + GOLDEN)  # counter 0 maps to state + GOLDEN

    def bits(self, idx: torch.Tensor) -> torch.Tensor:
        """64 random bits (as int64) for each counter in ``idx`` (int64)."""
        idx = idx.to(torch.int64)
        return mix64(idx * GOLDEN + self._first)

    def uniform(self, idx: torch.Tensor) -> torch.Tensor:
        """Doubles uniform on [0, 1): the top 53 bits times 2**-53."""
        return _srl(self.bits(idx), 11).to(torch.float64) * (2.0 ** -53)

    def randint(self, idx: torch.Tensor, bound: torch.Tensor | int) -> torch.Tensor:
        """Integers in [0, bound) by the multiply-shift map of the top 32 bits
        (Lemire, "Fast random integer generation in an interval", 2019,
        without the rejection step; the bias is below bound / 2**32)."""
        hi = _srl(self.bits(idx), 32)
        if isinstance(bound, int):
            assert 0 < bound < (1 << 31)
            return (hi * bound) >> 32
        return (hi * bound.to(torch.int64)) >> 32

    def normal(self, idx: torch.Tensor) -> torch.Tensor:
        """Standard normals by the Box-Muller transform of two uniforms
        drawn at counters 2*idx and 2*idx+1."""
        idx = idx.to(torch.int64)
        u1 = 1.0 - self.uniform(2 * idx)  # (0, 1]
        u2 = self.uniform(2 * idx + 1)
        return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos((2.0 * torch.pi) * u2)
