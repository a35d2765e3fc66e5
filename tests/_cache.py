"""Per-process cache of generated inputs and oracle results for the tests."""
import functools

from bse_synth import get, make_inputs


@functools.lru_cache(maxsize=8)
def inputs(name: str) -> dict:
    return make_inputs(get(name))


@functools.lru_cache(maxsize=8)
def oracle_run(name: str, bse_type: str = "singlet") -> dict:
    from oracle import bse_oracle as O
    return O.run(inputs(name), bse_type)
