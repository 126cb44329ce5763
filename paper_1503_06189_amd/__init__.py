"""MI355X-native X-engine correlator (4+4-bit complex, int8 MFMA).

Submodules:
  xengine  -- ctypes binding of libxengine.so (the HIP path)
  synth    -- seeded synthetic frames and loss masks
  metrics  -- rate and work definitions for reports
  tune     -- autotuner of batched persistent launches: tile geometry and
              time-chunk length, cached per device
  serve    -- streaming server: admission by HBM budget, continuous batching
"""

__version__ = "0.1.0"
