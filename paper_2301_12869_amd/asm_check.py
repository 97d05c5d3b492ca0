"""Build-time scan of generated gfx950 device assembly.

Rejects any code object that would write through the scalar data cache
(scalar stores, scalar atomics, scalar-cache write-back or discard): all
device writes in this library go through vector memory instructions.
This file only runs where the library is built.
"""
import re

_FORBIDDEN = re.compile(r"^\s*(s_store_|s_buffer_store|s_scratch_store|s_atomic|s_buffer_atomic|"
                        r"s_dcache_wb|s_dcache_discard)", re.M)


def scan(asm_text: str):
    return sorted(set(_FORBIDDEN.findall(asm_text)))
