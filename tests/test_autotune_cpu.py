"""Host logic of the autotuning cache (no GPU)."""
from paper_2502_15253_amd import autotune as AT
from paper_2502_15253_amd import synth


def test_tuning_key_separates_models_modes_devices_and_event_counts():
    d1, d3 = synth.config1_model(), synth.config3_model()
    k = AT.tuning_key(d1, [100000], "m64", "devA")
    assert k == AT.tuning_key(d1, [100000], "m64", "devA")
    others = [AT.tuning_key(d3, [100000], "m64", "devA"), AT.tuning_key(d1, [100001], "m64", "devA"),
              AT.tuning_key(d1, [100000], "m32", "devA"), AT.tuning_key(d1, [100000], "m64", "devB"),
              AT.tuning_key(d1, [100000], "m64", "devA", batch=64)]
    assert len(set(others + [k])) == 6
