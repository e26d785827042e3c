! CPU SIMD generation from Fortran (no GPU): reads a plain state blob of
! generator GEN from FILE_IN, makes a SIMD state from it, draws three single
! outputs and then N more with one fill, and writes the N + 3 words to
! FILE_OUT; also the next 5 values as doubles to FILE_OUT.f64.
!   simd_example GEN FILE_IN N FILE_OUT
program simd_example
  use iso_c_binding
  use prand
  implicit none
  integer(c_int) :: gen, rc
  integer(c_int64_t) :: n
  integer :: i, u
  character(len=1024) :: arg, fin, fout
  integer(c_int8_t), allocatable, target :: st(:), simd(:)
  integer(c_int32_t), allocatable, target :: out(:)
  real(c_double), target :: dbl(5)

  call get_command_argument(1, arg)
  read(arg, *) gen
  call get_command_argument(2, fin)
  call get_command_argument(3, arg)
  read(arg, *) n
  call get_command_argument(4, fout)

  allocate(st(prand_state_bytes(gen)))
  open(newunit=u, file=trim(fin), access='stream', form='unformatted', status='old')
  read(u) st
  close(u)

  allocate(simd(prand_simd_state_bytes()))
  rc = prand_get_simd_state(gen, c_loc(st), c_loc(simd))
  if (rc /= PRAND_OK) then
    print *, 'prand_get_simd_state: ', prand_strerror(rc)
    stop 1
  end if
  allocate(out(n + 3))
  do i = 1, 3
    out(i) = prand_simd_next(c_loc(simd))
  end do
  rc = prand_simd_fill(c_loc(simd), PRAND_U32, c_loc(out(4)), n)
  if (rc /= PRAND_OK) stop 2
  rc = prand_simd_fill(c_loc(simd), PRAND_F64, c_loc(dbl), 5_c_int64_t)
  if (rc /= PRAND_OK) stop 3
  ! a bad output type is refused with PRAND_EINVAL
  if (prand_simd_fill(c_loc(simd), 7_c_int, c_loc(dbl), 1_c_int64_t) /= PRAND_EINVAL) stop 4

  open(newunit=u, file=trim(fout), access='stream', form='unformatted', status='replace')
  write(u) out
  close(u)
  open(newunit=u, file=trim(fout)//'.f64', access='stream', form='unformatted', status='replace')
  write(u) dbl
  close(u)
end program simd_example
