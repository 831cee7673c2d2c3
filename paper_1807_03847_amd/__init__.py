"""MI355X (gfx950) certified top-k Katz ranking: HIP kernels behind the C ABI of
``include/katz.h`` and a thin ctypes binding (``paper_1807_03847_amd.katz``)."""
