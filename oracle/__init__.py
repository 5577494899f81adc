"""CPU oracle for the modified no-search (MNS) fractal encoder and its decoder.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constant generators).

Every function here is a plain, slow, direct restatement of the method in
"A Modified No Search Algorithm for Fractal Image Compression" (Salarian,
Mohamadinia, Rasekhi): integers (numpy int64) for encoding, float64 where
the decoder's definition is real-valued.  Readings of points the paper leaves
open are stated where they are used.

Modules:
  mns         -- the MNS encoder (Sec. 3, Sec. 3.1-3.3) and the record format
  fullsearch  -- the exhaustive range-domain search baseline (Sec. 1)
  decode      -- iterated-function-system decoding (Sec. 1)
  metrics     -- PSNR / MSE (Sec. 4)
"""
