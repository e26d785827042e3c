! prand.f90 -- Fortran bindings of the C ABI in prand.h (the paper's
! "Fortran compatibility": the library is callable from Fortran).
!
! Every interface below is the C function of the same name, through
! ISO_C_BINDING: states, outputs and contexts are passed as C addresses
! (c_loc of a TARGET array, or a type(c_ptr) handle), sizes and flags by
! value, 64-bit unsigned values (seeds, lengths, stream ids) as
! integer(c_int64_t) with the same bits.  Return codes are those of prand.h
! (PRAND_OK = 0, negative on error).  See prand.h for what each call does,
! its argument layout and ownership.
!
! Compile with the module first (e.g. amdflang -c prand.f90), then
! "use prand" and link against libprand.so.
module prand
  use iso_c_binding
  implicit none

  ! generators, output types, stream variants (prand.h enums)
  integer(c_int), parameter :: PRAND_MT19937 = 0, PRAND_MRG32K3A = 1, PRAND_LFSR113 = 2, &
                               PRAND_GM19 = 3, PRAND_GM29 = 4, PRAND_GM31 = 5, PRAND_GM55 = 6, &
                               PRAND_GM61 = 7, PRAND_GQ58X1 = 8, PRAND_GQ58X3 = 9, PRAND_GQ58X4 = 10
  integer(c_int), parameter :: PRAND_U32 = 0, PRAND_F32 = 1, PRAND_F64 = 2
  integer(c_int), parameter :: PRAND_SEQ_DEFAULT = 0, PRAND_SEQ = 1, PRAND_SEQ_SHORT = 2, &
                               PRAND_SEQ_MEDIUM = 3, PRAND_SEQ_LONG = 4
  integer(c_int), parameter :: PRAND_OK = 0, PRAND_EINVAL = -1, PRAND_EUNSUPPORTED = -2, &
                               PRAND_ERANGE = -3, PRAND_EHIP = -4, PRAND_ENOMEM = -5, &
                               PRAND_ENODEV = -6, PRAND_EBUSY = -7, PRAND_ENOTREADY = -8

  interface
    ! ---- metadata (host only)
    function prand_state_bytes(gen) bind(C, name="prand_state_bytes")
      import :: c_int, c_size_t
      integer(c_int), value :: gen
      integer(c_size_t) :: prand_state_bytes
    end function
    function prand_block_log2(gen, variant) bind(C, name="prand_block_log2")
      import :: c_int
      integer(c_int), value :: gen, variant
      integer(c_int) :: prand_block_log2
    end function
    function prand_independence_limit(gen, variant, streams, length) bind(C, name="prand_independence_limit")
      import :: c_int, c_double
      integer(c_int), value :: gen, variant
      real(c_double) :: streams, length
      integer(c_int) :: prand_independence_limit
    end function
    function prand_strerror_c(code) bind(C, name="prand_strerror")
      import :: c_int, c_ptr
      integer(c_int), value :: code
      type(c_ptr) :: prand_strerror_c
    end function

    ! ---- context
    function prand_ctx_create(ctx, hip_device) bind(C, name="prand_ctx_create")
      import :: c_int, c_ptr
      type(c_ptr) :: ctx
      integer(c_int), value :: hip_device
      integer(c_int) :: prand_ctx_create
    end function
    function prand_ctx_destroy(ctx) bind(C, name="prand_ctx_destroy")
      import :: c_int, c_ptr
      type(c_ptr), value :: ctx
      integer(c_int) :: prand_ctx_destroy
    end function

    ! ---- states on the host (rng_init_, rng_skipahead_, rng_init_*sequence_)
    function prand_init_default(ctx, gen, h_state) bind(C, name="prand_init_default")
      import :: c_int, c_ptr
      type(c_ptr), value :: ctx, h_state
      integer(c_int), value :: gen
      integer(c_int) :: prand_init_default
    end function
    function prand_seed(ctx, gen, seed, h_state) bind(C, name="prand_seed")
      import :: c_int, c_int64_t, c_ptr
      type(c_ptr), value :: ctx, h_state
      integer(c_int), value :: gen
      integer(c_int64_t), value :: seed
      integer(c_int) :: prand_seed
    end function
    function prand_skipahead(ctx, gen, h_state, h_dist, nlimbs) bind(C, name="prand_skipahead")
      import :: c_int, c_ptr
      type(c_ptr), value :: ctx, h_state, h_dist
      integer(c_int), value :: gen, nlimbs
      integer(c_int) :: prand_skipahead
    end function
    function prand_seed_host(gen, seed, h_state) bind(C, name="prand_seed_host")
      import :: c_int, c_int64_t, c_ptr
      type(c_ptr), value :: h_state
      integer(c_int), value :: gen
      integer(c_int64_t), value :: seed
      integer(c_int) :: prand_seed_host
    end function
    function prand_init_default_host(gen, h_state) bind(C, name="prand_init_default_host")
      import :: c_int, c_ptr
      type(c_ptr), value :: h_state
      integer(c_int), value :: gen
      integer(c_int) :: prand_init_default_host
    end function
    function prand_init_stream(ctx, gen, variant, id, h_state) bind(C, name="prand_init_stream")
      import :: c_int, c_int64_t, c_ptr
      type(c_ptr), value :: ctx, h_state
      integer(c_int), value :: gen, variant
      integer(c_int64_t), value :: id
      integer(c_int) :: prand_init_stream
    end function

    ! ---- generation (rng_generate_gpu_array_*, rng_generate_array_)
    function prand_generate(ctx, gen, h_state, dtype, d_out, n, stream) bind(C, name="prand_generate")
      import :: c_int, c_int64_t, c_ptr
      type(c_ptr), value :: ctx, h_state, d_out, stream
      integer(c_int), value :: gen, dtype
      integer(c_int64_t), value :: n
      integer(c_int) :: prand_generate
    end function
    function prand_generate_array(ctx, gen, h_state, dtype, h_out, n) bind(C, name="prand_generate_array")
      import :: c_int, c_int64_t, c_ptr
      type(c_ptr), value :: ctx, h_state, h_out
      integer(c_int), value :: gen, dtype
      integer(c_int64_t), value :: n
      integer(c_int) :: prand_generate_array
    end function
    function prand_generate_streams(ctx, gen, d_states, count, n_per_stream, dtype, d_out, stream) &
        bind(C, name="prand_generate_streams")
      import :: c_int, c_int32_t, c_int64_t, c_ptr
      type(c_ptr), value :: ctx, d_states, d_out, stream
      integer(c_int), value :: gen, dtype
      integer(c_int32_t), value :: count
      integer(c_int64_t), value :: n_per_stream
      integer(c_int) :: prand_generate_streams
    end function

    ! ---- CPU SIMD generation (rng_get_sse_state_, rng_sse_generate_)
    function prand_simd_state_bytes() bind(C, name="prand_simd_state_bytes")
      import :: c_size_t
      integer(c_size_t) :: prand_simd_state_bytes
    end function
    function prand_get_simd_state(gen, h_state, simd_state) bind(C, name="prand_get_simd_state")
      import :: c_int, c_ptr
      integer(c_int), value :: gen
      type(c_ptr), value :: h_state, simd_state
      integer(c_int) :: prand_get_simd_state
    end function
    ! the 32-bit output, returned with its bits in an integer(c_int32_t)
    function prand_simd_next(simd_state) bind(C, name="prand_simd_next")
      import :: c_int32_t, c_ptr
      type(c_ptr), value :: simd_state
      integer(c_int32_t) :: prand_simd_next
    end function
    function prand_simd_fill(simd_state, dtype, h_out, n) bind(C, name="prand_simd_fill")
      import :: c_int, c_int64_t, c_ptr
      type(c_ptr), value :: simd_state, h_out
      integer(c_int), value :: dtype
      integer(c_int64_t), value :: n
      integer(c_int) :: prand_simd_fill
    end function
    function prand_simd_vectorized(simd_state) bind(C, name="prand_simd_vectorized")
      import :: c_int, c_ptr
      type(c_ptr), value :: simd_state
      integer(c_int) :: prand_simd_vectorized
    end function
  end interface

contains

  ! prand_strerror as a Fortran string
  function prand_strerror(code) result(msg)
    integer(c_int), intent(in) :: code
    character(len=:), allocatable :: msg
    character(kind=c_char), pointer :: p(:)
    integer :: n
    interface
      function strlen(s) bind(C, name="strlen")
        import :: c_ptr, c_size_t
        type(c_ptr), value :: s
        integer(c_size_t) :: strlen
      end function
    end interface
    type(c_ptr) :: cp
    cp = prand_strerror_c(code)
    n = int(strlen(cp))
    call c_f_pointer(cp, p, [n])
    allocate(character(len=n) :: msg)
    msg = transfer(p(1:n), msg)
  end function

end module prand
