"""MI355X HDG-IMEX hot path: C-ABI library libhdg.so (HIP, gfx950) and its
ctypes binding.  Import ``paper_2410_09790_amd.hdg`` for the binding."""
